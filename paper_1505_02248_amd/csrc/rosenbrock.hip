// Exponential Rosenbrock-Euler LEM steps for the periodic viscous Burgers
// equation u_t = -(u^2/2)_x + nu u_xx (sections 3 and 4.2; gfx950).
//
//   u^{n+1} = u^n + dt phi_1(dt J_M) F(u^n)_M   on every region M_i, core rows
//
// J is the Jacobian of the centered discretization
//   F_i = -(u_{i+1}^2 - u_{i-1}^2)/(4 dx) + nu (u_{i+1} - 2 u_i + u_{i-1})/dx^2,
// frozen at the state of the last refresh; J_M is its principal submatrix on
// the box (couplings to outside nodes dropped; the whole-grid box D = 1 keeps
// the periodic coupling).  Each (block, ensemble member) has its own J_M: at a
// refresh the augmented matrices [[dt J_M, I], [0, 0]] of all of them are
// assembled here and exponentiated in one batch by the dense Pade pipeline;
// the core rows of the top-right block, phi_1(dt J_M), are kept.  A step is
// then F on the grid and one contraction per (block, member, core row).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

struct EreBox {
  int ox, h, cx, whole;  // core origin and size, buffer width, 1: box = periodic grid
};

__device__ __forceinline__ int ere_wrap(int a, int n) {
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// [[dt J_M, I], [0, 0]] for matrix u = blk * ns + s, row-major (2 nl)^2.
__global__ void ere_assemble_kernel(const double* __restrict__ x, const EreBox* boxes, int nb,
                                    int ns, int nl, int n, double dt, double dx, double nu,
                                    double* A) {
  const int n2 = 2 * nl;
  const int64_t per = (int64_t)n2 * n2;
  const int64_t total = per * nb * ns;
  const double d = nu / (dx * dx), a = 1.0 / (2.0 * dx);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = e / per;
    const int64_t rc = e - u * per;
    const int r = (int)(rc / n2), c = (int)(rc - (int64_t)r * n2);
    const int blk = (int)(u / ns), s = (int)(u - (int64_t)blk * ns);
    const EreBox b = boxes[blk];
    double v = 0.0;
    if (r < nl && c >= nl) {
      v = (c - nl == r) ? 1.0 : 0.0;
    } else if (r < nl) {
      // local neighbours of r; the whole-grid box wraps around
      const int lm = r > 0 ? r - 1 : (b.whole ? nl - 1 : -1);
      const int lp = r < nl - 1 ? r + 1 : (b.whole ? 0 : -1);
      if (c == r) {
        v = -2.0 * d;
      } else if (c == lm) {
        v = x[(int64_t)ere_wrap(b.ox - b.h + lm, n) * ns + s] * a + d;
      } else if (c == lp) {
        v = -x[(int64_t)ere_wrap(b.ox - b.h + lp, n) * ns + s] * a + d;
      }
      v *= dt;  // (nl >= 3: the two neighbours are distinct)
    }
    A[e] = v;
  }
}

// Phi[blk][row][l][s] = R[u][h + row][nl + l] (state fastest, for the step).
__global__ void ere_extract_kernel(const double* __restrict__ R, const EreBox* boxes, int nb,
                                   int ns, int nl, int rows, double* Phi) {
  const int n2 = 2 * nl;
  const int64_t total = (int64_t)nb * rows * nl * ns;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e % ns);
    int64_t t = e / ns;
    const int l = (int)(t % nl);
    t /= nl;
    const int row = (int)(t % rows);
    const int blk = (int)(t / rows);
    const int64_t u = (int64_t)blk * ns + s;
    Phi[e] = R[u * n2 * n2 + (int64_t)(boxes[blk].h + row) * n2 + nl + l];
  }
}

// f = dt F(x) on the periodic grid, state fastest.
__global__ void ere_rhs_kernel(const double* __restrict__ x, double* f, int n, int ns, double dt,
                               double dx, double nu) {
  const int64_t total = (int64_t)n * ns;
  const double d = nu / (dx * dx), a = 1.0 / (4.0 * dx);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ns), s = (int)(e - (int64_t)i * ns);
    const double u0 = x[e];
    const double um = x[(int64_t)(i == 0 ? n - 1 : i - 1) * ns + s];
    const double up = x[(int64_t)(i == n - 1 ? 0 : i + 1) * ns + s];
    f[e] = dt * (-(up * up - um * um) * a + (up - 2.0 * u0 + um) * d);
  }
}

// y(core) = x(core) + sum_l Phi[blk][row][l][s] f(gather(l), s).  One
// workgroup per (block, core row, 64 members): wave q of the four sums the
// local rows l = q, q + 4, ... for its 64 consecutive members (coalesced loads
// of Phi and f), the four partial sums meet in LDS.
__global__ __launch_bounds__(256) void ere_apply_kernel(const double* __restrict__ x,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ Phi,
                                                        const EreBox* boxes, int ns, int nl,
                                                        int rows, int n, double* y) {
  __shared__ double part[3][64];
  const int sch = (ns + 63) / 64;
  const int64_t t = blockIdx.x / sch;  // block * rows + row
  const int s = (int)(blockIdx.x - t * sch) * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;
  const int row = (int)(t % rows);
  const int blk = (int)(t / rows);
  const EreBox b = boxes[blk];
  double acc = 0.0;
  if (s < ns) {
    const double* ph = Phi + (t * nl) * ns + s;
    double a0 = 0.0, a1 = 0.0;
    int l = q;
    for (; l + 4 < nl; l += 8) {
      a0 = fma(ph[(int64_t)l * ns], f[(int64_t)ere_wrap(b.ox - b.h + l, n) * ns + s], a0);
      a1 = fma(ph[(int64_t)(l + 4) * ns], f[(int64_t)ere_wrap(b.ox - b.h + l + 4, n) * ns + s], a1);
    }
    if (l < nl) a0 = fma(ph[(int64_t)l * ns], f[(int64_t)ere_wrap(b.ox - b.h + l, n) * ns + s], a0);
    acc = a0 + a1;
  }
  if (q > 0) part[q - 1][threadIdx.x & 63] = acc;
  __syncthreads();
  if (q == 0 && s < ns) {
    const int i = threadIdx.x;
    const int64_t o = (int64_t)(b.ox + row) * ns + s;
    y[o] = x[o] + ((acc + part[0][i]) + (part[1][i] + part[2][i]));
  }
}

// phi_1(dt J_M) for boxes of nl <= 80 points, one workgroup per (block,
// member).  J_M is tridiagonal (periodic tridiagonal on the whole grid), so a
// product W X costs three FMAs per entry.  With W = dt J_M / 2^s scaled to
// |W|_1 <= 4:
//   F = phi_1(W) = sum_{k<=30} W^k / (k+1)!   (remainder below 4^31/32! ~ 2e-17)
// by Horner, F <- W F + I/(k+1)!, with F held in registers (each thread owns
// one column and MP/8 consecutive rows; the rows next to a thread's segment
// are exchanged through LDS), then E = e^W = I + W F and s doublings
//   phi_1(2W) = phi_1(W) (e^W + I) / 2,   e^{2W} = (e^W)^2
// (the last squaring is not needed): dense products on FP64 MFMA (16x16x4)
// over 16-padded tiles, row stride MP + 1 against LDS bank conflicts; every
// product is formed in registers and written after a barrier, so it may
// overwrite an operand.  Writes the core rows of F, contiguous per matrix,
// into P[blk * ns + s][row][l] and s into sq_out[blk * ns + s].
typedef double d4e __attribute__((ext_vector_type(4)));
constexpr int kPhiMaxN = 80;   // LDS: two 80 x 81 float64 matrices
constexpr int kPhiDeg = 30;    // Taylor degree
constexpr double kPhiTheta = 4.0;

struct InvFact {
  double c[kPhiDeg + 1];  // c[k] = 1 / (k+1)!
  constexpr InvFact() : c() {
    double v = 1.0;
    for (int k = 0; k <= kPhiDeg; ++k) { v /= (double)(k + 1); c[k] = v; }
  }
};
constexpr InvFact kInvFact;

template <int MP, int NT>
struct PhiTiles {
  static constexpr int nt = MP / 16, tiles = nt * nt, nw = NT / 64;
  static constexpr int tq = (tiles + nw - 1) / nw;  // tiles per wave (last may be absent)
  static constexpr int ld = MP + 1;
};

// acc[q] = (A B) on this wave's output tiles t = wave + q * nw
template <int MP, int NT>
__device__ __forceinline__ void phi_product(const double* A, const double* B,
                                            d4e (&acc)[PhiTiles<MP, NT>::tq]) {
  using T = PhiTiles<MP, NT>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool last = wv + (T::tq - 1) * T::nw < T::tiles;
  int ar[T::tq], bc[T::tq];
#pragma unroll
  for (int q = 0; q < T::tq; ++q) {
    const int t = wv + q * T::nw, ti = t / T::nt, tj = t - ti * T::nt;
    ar[q] = (ti * 16 + (lane & 15)) * T::ld + (lane >> 4);
    bc[q] = (lane >> 4) * T::ld + tj * 16 + (lane & 15);
    acc[q] = (d4e){0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int k0 = 0; k0 < MP; k0 += 4) {
#pragma unroll
    for (int q = 0; q < T::tq; ++q) {
      if (q < T::tq - 1 || last) {
        const double a = A[ar[q] + k0];
        const double b = B[bc[q] + k0 * T::ld];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
  }
}

// f(i, j, (A B)(i, j)) over this thread's entries of the product
template <int MP, int NT, typename Fn>
__device__ __forceinline__ void phi_store(const d4e (&acc)[PhiTiles<MP, NT>::tq], Fn f) {
  using T = PhiTiles<MP, NT>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool last = wv + (T::tq - 1) * T::nw < T::tiles;
#pragma unroll
  for (int q = 0; q < T::tq; ++q) {
    if (q < T::tq - 1 || last) {
      const int t = wv + q * T::nw, ti = t / T::nt, tj = t - ti * T::nt;
#pragma unroll
      for (int r = 0; r < 4; ++r) f(ti * 16 + 4 * r + (lane >> 4), tj * 16 + (lane & 15), acc[q][r]);
    }
  }
}

// Banded product on the register segment: out[m] = (W X)(r0 + m, j) + cdiag
// on the diagonal, X given by this thread's xs[] plus the exchanged rows.
// cl/cd/cu[m] are the entries W(i, i-1), W(i, i), W(i, i+1) of row i = r0 + m
// (i-1 and i+1 taken cyclically on the whole-grid box; zero where the box
// drops the coupling).
template <int RS, int MP>
__device__ __forceinline__ void band_step(const double (&xs)[RS], double (&out)[RS],
                                          const double (&cl)[RS], const double (&cd)[RS],
                                          const double (&cu)[RS], double* xch, double* lastrow,
                                          int r0, int seg, int j, int nl, bool whole,
                                          double cdiag) {
  // publish this segment's first and last rows and, if held here, row nl - 1
  xch[seg * MP + j] = xs[0];
  xch[(8 + seg) * MP + j] = xs[RS - 1];
#pragma unroll
  for (int m = 0; m < RS; ++m)
    if (r0 + m == nl - 1) lastrow[j] = xs[m];
  __syncthreads();
  const double prev = seg > 0 ? xch[(8 + seg - 1) * MP + j] : (whole ? lastrow[j] : 0.0);
  const double next = seg < 7 ? xch[(seg + 1) * MP + j] : 0.0;
  const double first = whole ? xch[j] : 0.0;  // row 0 (first row of segment 0)
#pragma unroll
  for (int m = 0; m < RS; ++m) {
    const int i = r0 + m;
    double v = (i == j) ? cdiag : 0.0;
    if (i < nl) {
      const double up = m > 0 ? xs[m > 0 ? m - 1 : 0] : prev;
      const double dn = (i == nl - 1) ? first : (m < RS - 1 ? xs[m < RS - 1 ? m + 1 : 0] : next);
      v += cl[m] * up + cd[m] * xs[m] + cu[m] * dn;
    }
    out[m] = v;
  }
}

// The same step when the box fills the tile (nl == MP): every row is live, the
// diagonal of W is one scalar, row nl - 1 is the last row of segment 7, and
// the identity term enters as an FMA with this thread's 0/1 diagonal mask em
// (one at the row equal to its column) instead of a compare and two selects.
template <int RS, int MP>
__device__ __forceinline__ void band_step_full(const double (&xs)[RS], double (&out)[RS],
                                               const double (&cl)[RS], double cd,
                                               const double (&cu)[RS], const double (&em)[RS],
                                               double* xch, int seg, int j, bool whole,
                                               double cdiag) {
  xch[seg * MP + j] = xs[0];
  xch[(8 + seg) * MP + j] = xs[RS - 1];
  __syncthreads();
  const double prev = seg > 0 ? xch[(8 + seg - 1) * MP + j] : (whole ? xch[15 * MP + j] : 0.0);
  const double next = seg < 7 ? xch[(seg + 1) * MP + j] : (whole ? xch[j] : 0.0);
#pragma unroll
  for (int m = 0; m < RS; ++m) {
    const double up = m > 0 ? xs[m > 0 ? m - 1 : 0] : prev;
    const double dn = m < RS - 1 ? xs[m < RS - 1 ? m + 1 : 0] : next;
    out[m] = fma(cl[m], up, fma(cd, xs[m], fma(cu[m], dn, em[m] * cdiag)));
  }
}

template <int MP, bool FULL>
__global__ __launch_bounds__(8 * MP) void ere_phi1_kernel(const double* __restrict__ x,
                                                          const EreBox* boxes, int ns, int nl,
                                                          int rows, int n, double dt, double dx,
                                                          double nu, double* P, int* sq_out,
                                                          int* status) {
  constexpr int NT = 8 * MP, RS = MP / 8;
  using T = PhiTiles<MP, NT>;
  constexpr int ld = T::ld, ms = MP * ld;
  extern __shared__ double sm[];
  double* F = sm;
  double* E = sm + ms;
  double* wl = sm + 2 * ms;  // W(i, im[i]), W(i, i), W(i, ip[i])
  double* wd = wl + MP;
  double* wu = wd + MP;
  double* xch = wu + MP;            // [parity][top 0..7 | bottom 8..15][MP]
  double* lastrow = xch + 32 * MP;  // [parity][MP]
  double* red = lastrow + 2 * MP;   // NT/64 partial maxima
  const int tid = threadIdx.x;
  const int j = tid % MP, seg = tid / MP, r0 = seg * RS;
  const int blk = blockIdx.x / ns, s = blockIdx.x - blk * ns;
  const EreBox b = boxes[blk];
  const double d = nu / (dx * dx), a = 1.0 / (2.0 * dx);
  // bands of dt J_M
  if (tid < MP) {
    const int r = tid;
    int lm = -1, lp = -1;
    double vl = 0.0, vd = 0.0, vu = 0.0;
    if (r < nl) {
      lm = r > 0 ? r - 1 : (b.whole ? nl - 1 : -1);
      lp = r < nl - 1 ? r + 1 : (b.whole ? 0 : -1);
      vd = -2.0 * d * dt;
      if (lm >= 0) vl = (x[(int64_t)ere_wrap(b.ox - b.h + lm, n) * ns + s] * a + d) * dt;
      if (lp >= 0) vu = (-x[(int64_t)ere_wrap(b.ox - b.h + lp, n) * ns + s] * a + d) * dt;
    }
    wl[r] = vl; wd[r] = vd; wu[r] = vu;
  }
  __syncthreads();
  // |W|_1: column c holds W(c, c), W(c-1, c) = wu[c-1], W(c+1, c) = wl[c+1] and,
  // on the whole-grid box, the wrap-around entries W(nl-1, 0) = wu[nl-1] and
  // W(0, nl-1) = wl[0] (zero elsewhere)
  double cs = 0.0;
  if (tid < MP) {
    const int c = tid;
    double t = fabs(wd[c]);
    if (c >= 1 && c < nl) t += fabs(wu[c - 1]);
    if (c + 1 < nl) t += fabs(wl[c + 1]);
    if (c == 0) t += fabs(wu[nl - 1]);
    if (c == nl - 1) t += fabs(wl[0]);
    cs = t;
  }
  for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = cs;
  __syncthreads();
  double nrm = 0.0;
  for (int w = 0; w < NT / 64; ++w) nrm = fmax(nrm, red[w]);
  int sq = 0;
  if (nrm > kPhiTheta && nrm < 1e300) sq = min(40, (int)ceil(log2(nrm / kPhiTheta)));
  if (tid == 0) {
    sq_out[blockIdx.x] = sq;
    if (!(nrm < 1e300)) atomicOr(status, kStatusNonFinite);
  }
  const double scale = ldexp(1.0, -sq);
  // this thread's rows of W = dt J_M / 2^s, in registers for the whole recursion
  double cl[RS], cd[RS], cu[RS], em[RS];
#pragma unroll
  for (int m = 0; m < RS; ++m) {
    cl[m] = wl[r0 + m] * scale;
    cd[m] = wd[r0 + m] * scale;
    cu[m] = wu[r0 + m] * scale;
    em[m] = (r0 + m == j) ? 1.0 : 0.0;
  }
  const double cd0 = cd[0];  // full tile: the one diagonal value of W
  const bool whole = b.whole != 0;
  auto step = [&](const double (&xs)[RS], double (&out)[RS], int par, double cdiag) {
    if constexpr (FULL)
      band_step_full<RS, MP>(xs, out, cl, cd0, cu, em, xch + par * 16 * MP, seg, j, whole, cdiag);
    else
      band_step<RS, MP>(xs, out, cl, cd, cu, xch + par * 16 * MP, lastrow + par * MP, r0, seg,
                        j, nl, whole, cdiag);
  };
  // Horner: F = I/(q+1)!, then F <- W F + I/(k+1)! for k = q-1 .. 0, in pairs
  // of steps (f -> g -> f) so that no copies are needed
  static_assert(kPhiDeg % 2 == 0, "Horner steps are taken in pairs");
  double f[RS], g[RS];
#pragma unroll
  for (int m = 0; m < RS; ++m) f[m] = em[m] * kInvFact.c[kPhiDeg];
  for (int k = kPhiDeg - 1; k >= 1; k -= 2) {
    step(f, g, 0, kInvFact.c[k]);
    step(g, f, 1, kInvFact.c[k - 1]);
  }
  const int par = 0;
#pragma unroll
  for (int m = 0; m < RS; ++m) F[(r0 + m) * ld + j] = f[m];
  if (sq > 0) {
    // E = I + W F
    step(f, g, par, 1.0);
#pragma unroll
    for (int m = 0; m < RS; ++m) E[(r0 + m) * ld + j] = g[m];
    __syncthreads();
    d4e acc[T::tq], acc2[T::tq];
    for (int q = 0; q < sq; ++q) {
      const bool square = q + 1 < sq;  // wave-uniform
      phi_product<MP, NT>(F, E, acc);  // F e^W
      if (square) phi_product<MP, NT>(E, E, acc2);
      __syncthreads();
      phi_store<MP, NT>(acc, [&](int i, int c, double v) { F[i * ld + c] = 0.5 * (v + F[i * ld + c]); });
      if (square) phi_store<MP, NT>(acc2, [&](int i, int c, double v) { E[i * ld + c] = v; });
      __syncthreads();
    }
  } else {
    __syncthreads();
  }
  // core rows of F (coalesced: one contiguous rows x nl block per matrix)
  double* out = P + (int64_t)blockIdx.x * rows * nl;
  for (int e = tid; e < rows * nl; e += NT) {
    const int row = e / nl, l = e - row * nl;
    out[e] = F[(b.h + row) * ld + l];
  }
}

// Phi[blk][k][s] = P[blk * ns + s][k] for k < K: per block a (ns x K) -> (K x ns)
// transpose through 32 x 32 LDS tiles (so the step reads Phi member-fastest).
__global__ __launch_bounds__(256) void ere_transpose_kernel(const double* __restrict__ P, int ns,
                                                            int K, double* __restrict__ Phi) {
  __shared__ double t[32][33];
  const int blk = blockIdx.z;
  const int k0 = blockIdx.x * 32, s0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* in = P + (int64_t)blk * ns * K;
  double* o = Phi + (int64_t)blk * K * ns;
#pragma unroll
  for (int r = 0; r < 32; r += 8) {
    const int sm = s0 + ty + r, k = k0 + tx;
    if (sm < ns && k < K) t[ty + r][tx] = in[(int64_t)sm * K + k];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 32; r += 8) {
    const int k = k0 + ty + r, sm = s0 + tx;
    if (sm < ns && k < K) o[(int64_t)k * ns + sm] = t[tx][ty + r];
  }
}

template <int MP, bool FULL>
static hipError_t launch_phi1_shape(const double* x, const void* boxes, int nb, int ns, int nl,
                              int rows, int n, double dt, double dx, double nu, double* P,
                              int* sq_out, int* status, hipStream_t st) {
  constexpr int NT = 8 * MP;
  const size_t lds = ((size_t)2 * MP * (MP + 1) + 3 * MP + 34 * MP + NT / 64) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)ere_phi1_kernel<MP, FULL>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((ere_phi1_kernel<MP, FULL>), dim3((unsigned)(nb * ns)), dim3(NT), lds, st, x,
                     (const EreBox*)boxes, ns, nl, rows, n, dt, dx, nu, P, sq_out, status);
  return hipGetLastError();
}

// boxes that fill the tile (nl == MP) take the specialized Horner step
template <int MP>
static hipError_t launch_phi1(const double* x, const void* boxes, int nb, int ns, int nl,
                              int rows, int n, double dt, double dx, double nu, double* P,
                              int* sq_out, int* status, hipStream_t st) {
  if (nl == MP)
    return launch_phi1_shape<MP, true>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out,
                                       status, st);
  return launch_phi1_shape<MP, false>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out,
                                      status, st);
}

static inline dim3 ere_grid(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

size_t ere_box_size() { return sizeof(EreBox); }

int ere_phi1_max_n() { return kPhiMaxN; }

hipError_t ere_phi1(const double* x, const void* boxes, int nb, int ns, int nl, int rows, int n,
                    double dt, double dx, double nu, double* P, double* Phi, int* sq_out,
                    int* status, hipStream_t st) {
  if (nl < 3 || nl > kPhiMaxN || nb < 1 || ns < 1 || rows < 1 || rows > nl)
    return hipErrorInvalidValue;
  hipError_t e;
  switch ((nl + 15) / 16) {
    case 1: e = launch_phi1<16>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out, status, st); break;
    case 2: e = launch_phi1<32>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out, status, st); break;
    case 3: e = launch_phi1<48>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out, status, st); break;
    case 4: e = launch_phi1<64>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out, status, st); break;
    default: e = launch_phi1<80>(x, boxes, nb, ns, nl, rows, n, dt, dx, nu, P, sq_out, status, st); break;
  }
  if (e != hipSuccess) return e;
  const int K = rows * nl;
  hipLaunchKernelGGL(ere_transpose_kernel, dim3((unsigned)((K + 31) / 32), (unsigned)((ns + 31) / 32),
                     (unsigned)nb), dim3(256), 0, st, P, ns, K, Phi);
  return hipGetLastError();
}

void ere_box_fill(void* dst, int i, int ox, int h, int cx, int whole) {
  EreBox* b = (EreBox*)dst + i;
  b->ox = ox; b->h = h; b->cx = cx; b->whole = whole;
}

hipError_t ere_assemble(const double* x, const void* boxes, int nb, int ns, int nl, int n,
                        double dt, double dx, double nu, double* A, hipStream_t st) {
  hipLaunchKernelGGL(ere_assemble_kernel, ere_grid((int64_t)4 * nl * nl * nb * ns), dim3(256), 0,
                     st, x, (const EreBox*)boxes, nb, ns, nl, n, dt, dx, nu, A);
  return hipGetLastError();
}

hipError_t ere_extract(const double* R, const void* boxes, int nb, int ns, int nl, int rows,
                       double* Phi, hipStream_t st) {
  hipLaunchKernelGGL(ere_extract_kernel, ere_grid((int64_t)nb * rows * nl * ns), dim3(256), 0, st,
                     R, (const EreBox*)boxes, nb, ns, nl, rows, Phi);
  return hipGetLastError();
}

hipError_t ere_step(const double* x, double* f, const double* Phi, const void* boxes, int nb,
                    int ns, int nl, int rows, int n, double dt, double dx, double nu, double* y,
                    hipStream_t st) {
  hipLaunchKernelGGL(ere_rhs_kernel, ere_grid((int64_t)n * ns), dim3(256), 0, st, x, f, n, ns, dt,
                     dx, nu);
  const int64_t wgs = (int64_t)nb * rows * ((ns + 63) / 64);
  hipLaunchKernelGGL(ere_apply_kernel, dim3((unsigned)wgs), dim3(256), 0, st, x, f, Phi,
                     (const EreBox*)boxes, ns, nl, rows, n, y);
  return hipGetLastError();
}

}  // namespace lem
