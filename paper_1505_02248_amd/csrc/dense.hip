// Dense local exponentials and their application (gfx950).
//
// Sections 3 and 4 of the paper store the local matrices exp(dt A_{M_i}) (or
// phi) of small subdomains, computed once by Pade approximation with scaling
// and squaring, and reuse them every step.  Here:
//
//  plan time (float64 throughout):
//   assemble_kernel     dense dt*A_M of every distinct local operator
//   var_assemble_kernel the same from face arrays (variable coefficients)
//   dgemm_kernel        batched C = A B on FP64 MFMA (v_mfma_f64_16x16x4):
//                       the powers and polynomial products of the Pade
//                       [13/13] approximant (or of the Taylor alternative)
//                       and the squarings
//   lincomb_kernel      elementwise linear combinations of those powers
//   lu_* kernels        Pade: Q X = P by LU with partial pivoting (right-hand
//                       sides eliminated alongside), then back substitution
//   pack_kernel         core rows of exp(dt A_M) into MFMA fragment order,
//                       in float64, float32 and bf16 hi/mid/lo pieces
//
//  step time:
//   apply_*_kernel      Y_k = E[core, :] X_k for every block k at once: the
//                       B operand rows are gathered from the global state by
//                       the box (periodic wrap), the epilogue writes the core
//                       rows straight into the new state (fused scatter).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// --------------------------------------------------------------- assembly --

// One distinct local operator: box dims and stencil weights of dt*A.
struct DenseOp {
  double w0, wW, wE, wS, wN;
  int Lx, Ly;
};

__global__ void assemble_kernel(const DenseOp* ops, double* A, int nl) {
  const int u = blockIdx.y;
  const DenseOp o = ops[u];
  double* M = A + (int64_t)u * nl * nl;
  const int64_t total = (int64_t)nl * nl;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / nl), c = (int)(e - (int64_t)r * nl);
    const int ry = r / o.Lx, rx = r - ry * o.Lx;
    double v = 0.0;
    if (c == r) v = o.w0;
    else if (c == r - 1 && rx > 0) v = o.wW;
    else if (c == r + 1 && rx < o.Lx - 1) v = o.wE;
    else if (c == r - o.Lx && ry > 0) v = o.wS;
    else if (c == r + o.Lx && ry < o.Ly - 1) v = o.wN;
    M[e] = v;
  }
}

// Max column sum |.| per matrix (the 1-norm) -> norms[u].
__global__ void norm1_kernel(const double* A, int nl, double* norms) {
  const int u = blockIdx.x;
  const double* M = A + (int64_t)u * nl * nl;
  __shared__ double red[16];
  double best = 0.0;
  for (int c = threadIdx.x; c < nl; c += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < nl; ++r) s += fabs(M[(int64_t)r * nl + c]);
    best = fmax(best, s);
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = fmax(b, red[w]);
    norms[u] = b;
  }
}

// A <- A * 2^-s[u]
__global__ void scale_pow2_kernel(double* A, int nl, const int* s) {
  const int u = blockIdx.y;
  double* M = A + (int64_t)u * nl * nl;
  const int64_t total = (int64_t)nl * nl;
  const int e2 = -s[u];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    M[e] = ldexp(M[e], e2);
}

// out = c0 X0 + c1 X1 + c2 X2 + c3 X3 + d I  (any Xi may be null)
struct LinComb {
  const double* X[4];
  double c[4];
  double d;
  double* out;
  int nl;
  int64_t stride;  // matrix stride of every operand (batched)
};

__global__ void lincomb_kernel(LinComb p) {
  const int u = blockIdx.y;
  const int64_t off = (int64_t)u * p.stride;
  const int64_t total = (int64_t)p.nl * p.nl;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (p.X[q]) v = fma(p.c[q], p.X[q][off + e], v);
    const int r = (int)(e / p.nl);
    if (e - (int64_t)r * p.nl == r) v += p.d;
    p.out[off + e] = v;
  }
}

// P = V + U, Q = V - U (in place: V -> P, U -> Q)
__global__ void pade_pq_kernel(double* V, double* U, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = V[e], u = U[e];
    V[e] = v + u;
    U[e] = v - u;
  }
}

// ------------------------------------------------------------------ DGEMM --
// C[u] = A[u] * B[u], row-major nl x nl, FP64 MFMA 16x16x4.  64x64 tile per
// workgroup of 256 threads; each wave owns a 32x32 quarter (2x2 MFMA tiles).
// Fragment layouts (16x16x4, f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l is D[4*r + l/16][l%16]
// (the f32 and bf16 forms place it at D[4*(l/16) + r][l%16] instead).
__global__ __launch_bounds__(256) void dgemm_kernel(const double* A, const double* B,
                                                    double* C, int nl, int64_t stride) {
  constexpr int BM = 64, BK = 16;
  __shared__ double As[BM][BK + 1];
  __shared__ double Bs[BK][BM + 2];
  const int u = blockIdx.z;
  const double* Ab = A + (int64_t)u * stride;
  const double* Bb = B + (int64_t)u * stride;
  double* Cb = C + (int64_t)u * stride;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BM;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < nl; k0 += BK) {
    {  // A tile 64 x 16
      const int r = tid >> 2, c = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = m0 + r, gc = k0 + c + q;
        As[r][c + q] = (gr < nl && gc < nl) ? Ab[(int64_t)gr * nl + gc] : 0.0;
      }
    }
    {  // B tile 16 x 64
      const int r = tid >> 4, c = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = k0 + r, gc = n0 + c + q;
        Bs[r][c + q] = (gr < nl && gc < nl) ? Bb[(int64_t)gr * nl + gc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[wr + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bfr[j] = Bs[kk + (lane >> 4)][wc + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = m0 + wr + i * 16 + 4 * r + (lane >> 4);
        const int gc = n0 + wc + j * 16 + (lane & 15);
        if (gr < nl && gc < nl) Cb[(int64_t)gr * nl + gc] = acc[i][j][r];
      }
}

// ------------------------------------------------------------- LU solve --
// Solve Q X = P (batched, nl x nl, right-hand sides P overwritten by X).
// Column step j: choose the pivot row, swap it into row j in Q and P, store
// the multipliers l_ij = Q[i][j]/Q[j][j] in Q[i][j]; then eliminate below.
__global__ __launch_bounds__(256) void lu_pivot_kernel(double* Q, double* P, int nl,
                                                       int64_t stride, int j) {
  const int u = blockIdx.x;
  double* Qb = Q + (int64_t)u * stride;
  double* Pb = P + (int64_t)u * stride;
  __shared__ double bv[4];
  __shared__ int bi[4];
  __shared__ int sp;
  const int tid = threadIdx.x;
  double best = -1.0;
  int bidx = j;
  for (int i = j + tid; i < nl; i += 256) {
    const double a = fabs(Qb[(int64_t)i * nl + j]);
    if (a > best) { best = a; bidx = i; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bidx, off, 64);
    if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
  }
  if ((tid & 63) == 0) { bv[tid >> 6] = best; bi[tid >> 6] = bidx; }
  __syncthreads();
  if (tid == 0) {
    double b = bv[0];
    int p = bi[0];
    for (int w = 1; w < 4; ++w)
      if (bv[w] > b || (bv[w] == b && bi[w] < p)) { b = bv[w]; p = bi[w]; }
    sp = p;
  }
  __syncthreads();
  const int p = sp;
  if (p != j) {
    for (int k = tid; k < 2 * nl; k += 256) {
      double* M = k < nl ? Qb : Pb;
      const int kk = k < nl ? k : k - nl;
      const double t = M[(int64_t)j * nl + kk];
      M[(int64_t)j * nl + kk] = M[(int64_t)p * nl + kk];
      M[(int64_t)p * nl + kk] = t;
    }
    __syncthreads();
  }
  const double inv = 1.0 / Qb[(int64_t)j * nl + j];
  for (int i = j + 1 + tid; i < nl; i += 256) Qb[(int64_t)i * nl + j] *= inv;
}

// rows i > j: Q[i][k] -= l_ij Q[j][k] (k > j), P[i][k] -= l_ij P[j][k] (all k)
__global__ void lu_elim_kernel(double* Q, double* P, int nl, int64_t stride, int j) {
  const int u = blockIdx.z;
  double* Qb = Q + (int64_t)u * stride;
  double* Pb = P + (int64_t)u * stride;
  const int i = j + 1 + blockIdx.y;
  if (i >= nl) return;
  const double l = Qb[(int64_t)i * nl + j];
  const int qcols = nl - j - 1;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < qcols + nl;
       c += gridDim.x * blockDim.x) {
    if (c < qcols) {
      const int k = j + 1 + c;
      Qb[(int64_t)i * nl + k] = fma(-l, Qb[(int64_t)j * nl + k], Qb[(int64_t)i * nl + k]);
    } else {
      const int k = c - qcols;
      Pb[(int64_t)i * nl + k] = fma(-l, Pb[(int64_t)j * nl + k], Pb[(int64_t)i * nl + k]);
    }
  }
}

// back substitution step j: rows i < j: P[i][k] -= Q[i][j] * (P[j][k] / Q[j][j])
// (row j itself is divided by its pivot at the very end).
__global__ void lu_back_kernel(const double* Q, double* P, int nl, int64_t stride, int j) {
  const int u = blockIdx.z;
  const double* Qb = Q + (int64_t)u * stride;
  double* Pb = P + (int64_t)u * stride;
  const int i = blockIdx.y;
  if (i >= j) return;
  const double f = Qb[(int64_t)i * nl + j] / Qb[(int64_t)j * nl + j];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nl; k += gridDim.x * blockDim.x)
    Pb[(int64_t)i * nl + k] = fma(-f, Pb[(int64_t)j * nl + k], Pb[(int64_t)i * nl + k]);
}

__global__ void lu_diag_kernel(const double* Q, double* P, int nl, int64_t stride) {
  const int u = blockIdx.z;
  const double* Qb = Q + (int64_t)u * stride;
  double* Pb = P + (int64_t)u * stride;
  const int i = blockIdx.y;
  const double inv = 1.0 / Qb[(int64_t)i * nl + i];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nl; k += gridDim.x * blockDim.x)
    Pb[(int64_t)i * nl + k] *= inv;
}

// ------------------------------------------------------------------- pack --
// Core rows of R (nl x nl) -> fragment-ordered operands.  Rows R_core x cols
// K = nl are padded to multiples of 16 (rows) and 32 (cols) with zeros.
//  f64/f32: [rt][kk][lane]        = E[rt*16 + lane%16][kk*4 + lane/16]
//  bf16   : [piece][rt][ks][lane][e] = piece of E[rt*16 + lane%16][ks*32 + 8*(lane/16) + e]
struct PackArgs {
  const double* R;
  int nl, Lx, h, cx, cy, ndim;
  int rows, rows_p, cols_p;  // core rows, padded rows, padded cols
  double* e64;
  float* e32;
  __hip_bfloat16* e16;       // 3 pieces
  double* core_out;          // plain copy of the core rows [rows][nl] (may be null)
};

__device__ __forceinline__ int core_to_local(int r, int cx, int h, int Lx, int ndim) {
  if (ndim == 1) return h + r;
  const int ry = r / cx, rx = r - ry * cx;
  return (h + ry) * Lx + h + rx;
}

__global__ void pack_kernel(PackArgs a) {
  const int64_t total = (int64_t)a.rows_p * a.cols_p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / a.cols_p), c = (int)(e - (int64_t)r * a.cols_p);
    double v = 0.0;
    if (r < a.rows && c < a.nl) {
      const int lr = core_to_local(r, a.cx, a.h, a.Lx, a.ndim);
      v = a.R[(int64_t)lr * a.nl + c];
      if (a.core_out) a.core_out[(int64_t)r * a.nl + c] = v;
    }
    const int rt = r >> 4, ri = r & 15;
    {  // f64 / f32 fragments (k-step 4)
      const int kk = c >> 2, kq = c & 3;
      const int64_t idx = (((int64_t)rt * (a.cols_p >> 2) + kk) << 6) + (kq << 4) + ri;
      a.e64[idx] = v;
      if (a.e32) a.e32[idx] = (float)v;
    }
    if (a.e16) {  // bf16 pieces (k-step 32)
      const int ks = c >> 5, kr = c & 31;
      const int lane = ri + 16 * (kr >> 3), el = kr & 7;
      const int64_t idx = ((((int64_t)rt * (a.cols_p >> 5) + ks) << 6) + lane) * 8 + el;
      const int64_t piece = (int64_t)a.rows_p * a.cols_p;
      const __hip_bfloat16 hi = __double2bfloat16(v);
      const double r1 = v - (double)__bfloat162float(hi);
      const __hip_bfloat16 mid = __double2bfloat16(r1);
      const double r2 = r1 - (double)__bfloat162float(mid);
      const __hip_bfloat16 lo = __double2bfloat16(r2);
      a.e16[idx] = hi;
      a.e16[piece + idx] = mid;
      a.e16[2 * piece + idx] = lo;
    }
  }
}

// ------------------------------------------------------------------ apply --
// Block table entry of the dense apply: box and which stored block it uses.
struct DBlock {
  int ox, oy, cx, cy, h, Lx, Ly;
  int unique;
};

struct ApplyArgs {
  const DBlock* blocks;
  const void* E;        // packed operand (f64, f32 or bf16 pieces)
  int64_t e_stride;     // elements per stored block (per piece for bf16)
  const double* x_in;
  double* x_out;
  int n, ndim, ns;      // grid side, dimension, ensemble size
  int rows, rows_p, cols, cols_p;
  int n_blocks, row_tiles, col_tiles;
  const double* bias;   // added to every output (forced steps), or null
  const __bf16* xp;     // split-bf16 apply: the state split into pieces once per
                        // step, interleaved per entry (2 pieces: hi, mid; 3 pieces:
                        // hi, mid, lo, 0 -- 4 or 8 bytes per entry), or null
  int* status;          // latched status bits (non-finite outputs), or null
};

// Latches kStatusNonFinite when this lane wrote a non-finite value.
__device__ __forceinline__ void latch_nonfinite(bool bad, int* status) {
  if (bad && status) atomicOr(status, kStatusNonFinite);
}

__device__ __forceinline__ int64_t dense_gather(const DBlock& b, int l, int n, int ndim) {
  const int ly = l / b.Lx, lx = l - ly * b.Lx;
  const int gx = wrap(b.ox - b.h + lx, n);
  if (ndim == 1) return gx;
  const int gy = wrap(b.oy - b.h + ly, n);
  return (int64_t)gy * n + gx;
}

__device__ __forceinline__ int64_t dense_scatter(const DBlock& b, int r, int n, int ndim) {
  if (ndim == 1) return b.ox + r;
  const int ry = r / b.cx, rx = r - ry * b.cx;
  return (int64_t)(b.oy + ry) * n + b.ox + rx;
}

// XCD-aware order: consecutive workgroup ids are spread over the 8 XCDs, so
// give each XCD a contiguous range of (block, row tile) work items; spatially
// adjacent blocks then share their halo rows in one L2.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int per = total / 8, rem = total % 8;
  const int xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// FP64 / FP32 apply.  Workgroup = NW waves, tile = (NW*WM) core rows x 64
// states of one block; wave w owns rows [w*WM, (w+1)*WM).  The K loop runs
// over chunks of KC local rows:
//  * A fragments (packed E, L2-resident when all blocks share one stored
//    block) are prefetched one chunk ahead into registers;
//  * the gathered X rows of chunk c+2 are loaded into registers while chunk c
//    is multiplied, and written to the LDS stage of chunk c+1 after it, so a
//    gather has two chunks of MFMA time to arrive (two LDS stages, one
//    barrier per chunk);
//  * the B fragments of k-step kk+1 are read from LDS before the MFMAs of kk.
// Every load is unconditional (indices clamped: the padded columns of E are
// zero, so a clamped X row contributes nothing), which keeps the loop body
// free of branches around memory operations and lets the compiler count
// outstanding loads exactly.  The loop is unrolled by two so that register
// sets and LDS stages are addressed statically.  Lane l of a B fragment holds
// states 4*(l%16) .. 4*(l%16)+3 (one 32-byte LDS read, one 32-byte store).
template <typename T, int WM, int KC, int NW>
__global__ __launch_bounds__(64 * NW) void apply_mfma_kernel(ApplyArgs a) {
  constexpr int BN = 64, RT = WM / 16, CT = 4, KK = KC / 4;
  constexpr int XS = BN + 4;            // padded LDS row (keeps 32-byte alignment)
  constexpr int EPT = KC * BN / (64 * NW);  // X elements per thread per chunk
  constexpr int TPR = BN / EPT;         // threads per X row
  static_assert(EPT >= 1 && BN % EPT == 0, "X chunk does not tile the workgroup");
  __shared__ T Xs0[KC][XS], Xs1[KC][XS];
  typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;

  const int total = a.n_blocks * a.row_tiles * a.col_tiles;
  const int item = xcd_remap(blockIdx.x, total);
  const int ct0 = item % a.col_tiles;
  const int rest = item / a.col_tiles;
  const int rtile = rest % a.row_tiles;
  const int blk = rest / a.row_tiles;
  const DBlock b = a.blocks[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = rtile * NW * WM + wv * WM;  // first core row of this wave
  const int col0 = ct0 * BN;
  const int ksteps = a.cols_p >> 2;
  const bool wave_live = row0 < a.rows_p;
  // this wave's first fragment (row tile row0/16, k-step 0, this lane); waves
  // past the padded rows read row tile 0 and discard it
  const T* Ew = reinterpret_cast<const T*>(a.E) + (int64_t)b.unique * a.e_stride +
                ((int64_t)(wave_live ? row0 >> 4 : 0) * ksteps << 6) + lane;
  const int64_t rt_stride = (int64_t)ksteps << 6;
  const int nchunks = a.cols_p / KC;
  const int last = nchunks - 1;

  acc_t acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  auto load_a = [&](int ch, T (&af)[KK][RT]) {
    const T* src = Ew + ((int64_t)ch * KK << 6);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
      for (int i = 0; i < RT; ++i) af[kk][i] = src[i * rt_stride + (kk << 6)];
  };
  const int xr = tid / TPR, xc = (tid % TPR) * EPT;
  auto load_x = [&](int ch, double (&v)[EPT]) {
    int l = ch * KC + xr;
    l = l < a.cols ? l : a.cols - 1;
    const int64_t g = dense_gather(b, l, a.n, a.ndim);
    const double* src = a.x_in + g * a.ns + col0 + xc;
#pragma unroll
    for (int q = 0; q < EPT; ++q) v[q] = src[q];
  };
  auto store_x = [&](const double (&v)[EPT], T (*X)[XS]) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) X[xr][xc + q] = (T)v[q];
  };
  auto mfma_chunk = [&](T (&af)[KK][RT], T (*X)[XS]) {
    T bb[2][CT];
    auto rd = [&](int kk, T (&bfr)[CT]) {
      const T* p = &X[kk * 4 + (lane >> 4)][(lane & 15) * 4];
#pragma unroll
      for (int j = 0; j < CT; ++j) bfr[j] = p[j];
    };
    rd(0, bb[0]);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      if (kk + 1 < KK) rd(kk + 1, bb[(kk + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);  // keep the next reads ahead of these MFMAs
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          if constexpr (sizeof(T) == 8)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk][i], bb[kk & 1][j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kk][i], bb[kk & 1][j], acc[i][j], 0, 0, 0);
        }
    }
  };
  // chunk c: multiply (acur, Xc); prefetch A of c+1 into anext and X of c+2
  // into xcur; then stage X of c+1 (xnext, loaded one chunk earlier) into Xn
  auto step = [&](int c, T (&acur)[KK][RT], T (&anext)[KK][RT], T (*Xc)[XS], T (*Xn)[XS],
                  double (&xcur)[EPT], double (&xnext)[EPT]) {
    load_a(c + 1 < last ? c + 1 : last, anext);
    load_x(c + 2 < last ? c + 2 : last, xcur);
    if (wave_live) mfma_chunk(acur, Xc);
    store_x(xnext, Xn);
    __syncthreads();
  };

  T a0[KK][RT], a1[KK][RT];
  double x0[EPT], x1[EPT];
  load_a(0, a0);
  load_x(0, x0);
  load_x(last < 1 ? last : 1, x1);
  store_x(x0, Xs0);
  __syncthreads();
  int c = 0;
  for (; c + 1 < nchunks; c += 2) {
    step(c, a0, a1, Xs0, Xs1, x0, x1);
    step(c + 1, a1, a0, Xs1, Xs0, x1, x0);
  }
  if (c < nchunks) step(c, a0, a1, Xs0, Xs1, x0, x1);

  if (!wave_live) return;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // accumulator row: f64 16x16x4 interleaves rows across registers
      const int tr = (sizeof(T) == 8) ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
      const int row = row0 + i * 16 + tr;
      if (row >= a.rows) continue;
      const int64_t g = dense_scatter(b, row, a.n, a.ndim);
      const int64_t o = g * a.ns + col0 + (lane & 15) * 4;
      double* dst = a.x_out + o;
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        const double v = (double)acc[i][j][r] + (a.bias ? a.bias[o + j] : 0.0);
        bad |= !isfinite(v);
        dst[j] = v;
      }
    }
  latch_nonfinite(bad, a.status);
}

// Split-bf16 apply: E = E_hi + E_mid + E_lo and X = X_hi + X_mid + X_lo are
// multiplied term by term on bf16 MFMA (16x16x32) with float32 accumulation.
// NT = 3 uses hi*hi + hi*lo' + lo'*hi with 2-piece operands (lo' = mid);
// NT = 6 adds hi*lo + lo*hi + mid*mid of the 3-piece split.
// Fragment layout (16x16x32 bf16): lane l supplies A[l%16][8*(l/16) + e] and
// B[8*(l/16) + e][l%16] for e = 0..7.
//
// The gathered row offsets of the box are tabulated in LDS once.  Thread t
// stages column t % 64 of k-group t / 64 (8 consecutive local rows) of the
// next chunk: eight coalesced loads, the split into pieces (float conversions:
// any bf16 close to the value serves as a piece, the residuals are exact), and
// one 16-byte LDS store per piece, into the LDS stage the MFMAs are not
// reading (one barrier per chunk).  A fragments are prefetched one chunk ahead.
__device__ __forceinline__ __bf16 bf16_near(double v) { return (__bf16)(float)v; }
__device__ __forceinline__ double bf16_val(__bf16 h) { return (double)(float)h; }

// The state split into bf16 pieces once per step (the apply kernels of every
// row tile of a block then only gather and pack them): x = hi + mid + lo with
// hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), the same split
// the apply performs when no pieces are given.  The pieces of an entry are
// adjacent (one 4- or 8-byte load brings all of them).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <int NP>
__global__ void split_pieces_kernel(const double* __restrict__ x, int64_t total,
                                    typename std::conditional<NP == 3, bf16x4, bf16x2>::type* P) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[e];
    const __bf16 hi = (__bf16)(float)v;
    const double r1 = v - (double)(float)hi;
    const __bf16 mid = (__bf16)(float)r1;
    if constexpr (NP == 3) {
      bf16x4 o;
      o[0] = hi; o[1] = mid; o[2] = (__bf16)(float)(r1 - (double)(float)mid); o[3] = (__bf16)0.0f;
      P[e] = o;
    } else {
      bf16x2 o;
      o[0] = hi; o[1] = mid;
      P[e] = o;
    }
  }
}

// BN states per workgroup: 64, or 128 (each stored-block fragment then feeds
// twice the MFMAs, halving the stored-block traffic per product; the gathered
// row offsets are then kept as 32-bit grid points to leave LDS for two
// workgroups per CU).
template <int NTERMS, int WM, int NW, bool PRE, int BN>
__global__ __launch_bounds__(64 * NW) void apply_bf16_kernel(ApplyArgs a) {
  constexpr int KC = 32, RT = WM / 16, CT = BN / 16;
  constexpr int NP = NTERMS == 6 ? 3 : 2;  // operand pieces in use
  constexpr int KG = KC / 8 + 1;           // padded k-groups per LDS column
  constexpr int GROUPS = 64 * NW / BN;     // thread groups staging one column each
  constexpr int KPT = KC / GROUPS;         // staged rows per thread (8 or 4)
  static_assert(NW == 4 || NW == 8, "four or eight waves");
  static_assert(KPT == 4 || KPT == 8, "four or eight staged rows per thread");
  __shared__ bf16x8 Xs[2][NP][BN][KG];
  // gathered rows of the chunk: element offsets g ns + col0 (64 states per
  // workgroup) or grid points g (128 states; offsets formed at the load)
  typedef typename std::conditional<BN == 128, int, int64_t>::type goff_t;
  extern __shared__ int64_t goff_raw[];
  goff_t* goff = reinterpret_cast<goff_t*>(goff_raw);
  const int total = a.n_blocks * a.row_tiles * a.col_tiles;
  const int item = xcd_remap(blockIdx.x, total);
  const int ct0 = item % a.col_tiles;
  const int rest = item / a.col_tiles;
  const int rtile = rest % a.row_tiles;
  const int blk = rest / a.row_tiles;
  const DBlock b = a.blocks[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = rtile * NW * WM + wv * WM;
  const int col0 = ct0 * BN;
  const bf16x8* E = reinterpret_cast<const bf16x8*>(a.E);
  const int64_t estride8 = a.e_stride / 8;  // per piece, in 8-element groups
  const int ksteps = a.cols_p >> 5;
  const bool wave_live = row0 < a.rows_p;
  const int rtw = wave_live ? row0 >> 4 : 0;
  const bf16x8* Ew = E + (int64_t)b.unique * 3 * estride8 + (int64_t)rtw * ksteps * 64 + lane;
  for (int l = tid; l < a.cols_p; l += 64 * NW) {
    const int lc = l < a.cols ? l : a.cols - 1;  // padded columns of E are zero
    if constexpr (BN == 128)
      goff[l] = (int)dense_gather(b, lc, a.n, a.ndim);
    else
      goff[l] = dense_gather(b, lc, a.n, a.ndim) * a.ns + col0;
  }
  __syncthreads();

  f4 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  auto load_a = [&](int ch, bf16x8 (&ea)[NP][RT]) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < RT; ++i)
        ea[p][i] = Ew[p * estride8 + ((int64_t)i * ksteps + ch) * 64];
  };
  const int xc = tid % BN, xg = tid / BN;
  // staged X of one chunk: KPT local rows of column xc, as float64 values
  // (split here) or as pieces (split once per step by split_pieces_kernel)
  typedef typename std::conditional<NP == 3, bf16x4, bf16x2>::type piece_t;
  typedef typename std::conditional<PRE, piece_t[KPT], double[KPT]>::type xreg_t;
  auto x_at = [&](int l) -> int64_t {
    if constexpr (BN == 128)
      return (int64_t)goff[l] * a.ns + col0 + xc;
    else
      return goff[l] + xc;
  };
  auto load_x = [&](int ch, xreg_t& v) {
    if constexpr (PRE) {
      const piece_t* xp = reinterpret_cast<const piece_t*>(a.xp);
#pragma unroll
      for (int e = 0; e < KPT; ++e) v[e] = xp[x_at(ch * KC + xg * KPT + e)];
    } else {
#pragma unroll
      for (int e = 0; e < KPT; ++e) v[e] = a.x_in[x_at(ch * KC + xg * KPT + e)];
    }
  };
  // rows xg*KPT .. xg*KPT + KPT - 1 of the chunk land in k-group xg*KPT/8
  // (all of it with eight rows per thread, one half of it with four)
  auto put = [&](int buf, int p, const bf16x8& v) {
    if constexpr (KPT == 8) {
      Xs[buf][p][xc][xg] = v;
    } else {
      bf16x4 h4;
#pragma unroll
      for (int e = 0; e < 4; ++e) h4[e] = v[e];
      reinterpret_cast<bf16x4*>(&Xs[buf][p][xc][xg >> 1])[xg & 1] = h4;
    }
  };
  auto store_x = [&](const xreg_t& v, int buf) {
    if constexpr (PRE) {
      bf16x8 pc[NP];
#pragma unroll
      for (int e = 0; e < KPT; ++e)
#pragma unroll
        for (int p = 0; p < NP; ++p) pc[p][e] = v[e][p];
#pragma unroll
      for (int p = 0; p < NP; ++p) put(buf, p, pc[p]);
    } else {
      bf16x8 pc[NP];
#pragma unroll
      for (int e = 0; e < KPT; ++e) {
        const __bf16 hi = bf16_near(v[e]);
        const double r1 = v[e] - bf16_val(hi);
        const __bf16 mid = bf16_near(r1);
        pc[0][e] = hi;
        pc[1][e] = mid;
        if constexpr (NP == 3) pc[2][e] = bf16_near(r1 - bf16_val(mid));
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) put(buf, p, pc[p]);
    }
  };
  auto mfma_chunk = [&](const bf16x8 (&ea)[NP][RT], int buf) {
    bf16x8 bx[NP][CT];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int j = 0; j < CT; ++j) bx[p][j] = Xs[buf][p][j * 16 + (lane & 15)][lane >> 4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        f4 c = acc[i][j];
        // small terms first, the dominant product last
        if constexpr (NTERMS == 6) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[1][i], bx[1][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[2][i], bx[0][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[0][i], bx[2][j], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[1][i], bx[0][j], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[0][i], bx[1][j], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ea[0][i], bx[0][j], c, 0, 0, 0);
        acc[i][j] = c;
      }
  };
  const int last = ksteps - 1;
  bf16x8 ea0[NP][RT], ea1[NP][RT];
  xreg_t xv;
  load_a(0, ea0);
  load_x(0, xv);
  store_x(xv, 0);
  __syncthreads();
  // chunk c in stage c & 1: prefetch A of c+1 and X of c+1, multiply, then
  // split and stage X of c+1 into the other stage; loads are unconditional
  // (clamped) so the loop body has no branches around memory operations
  auto step = [&](int c, const bf16x8 (&ecur)[NP][RT], bf16x8 (&enext)[NP][RT]) {
    const int cn = c + 1 < last ? c + 1 : last;
    load_a(cn, enext);
    load_x(cn, xv);
    if (wave_live) mfma_chunk(ecur, c & 1);
    store_x(xv, (c + 1) & 1);
    __syncthreads();
  };
  int c = 0;
  for (; c + 1 < ksteps; c += 2) {
    step(c, ea0, ea1);
    step(c + 1, ea1, ea0);
  }
  if (c < ksteps) step(c, ea0, ea1);

  if (!wave_live) return;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + i * 16 + 4 * (lane >> 4) + r;
      if (row >= a.rows) continue;
      const int64_t g = dense_scatter(b, row, a.n, a.ndim);
      const int64_t o = g * a.ns + col0 + (lane & 15);
      double* dst = a.x_out + o;
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        const double v = (double)acc[i][j][r] + (a.bias ? a.bias[o + j * 16] : 0.0);
        bad |= !isfinite(v);
        dst[j * 16] = v;
      }
    }
  latch_nonfinite(bad, a.status);
}

// Small ensembles (ns not a multiple of 64): eight lanes per (core row, state)
// with the plain row-major core block, float64 or float32 arithmetic.
template <typename T>
__global__ void apply_simple_kernel(ApplyArgs a, const double* core) {
  // LS lanes per output: lane p of a group takes the terms l = p, p + LS, ...
  // with four independent partial sums, then the group adds its lanes (groups
  // are aligned LS-lane slices of a wave, all active or all inactive)
  constexpr int LS = 8;
  const int64_t outputs = (int64_t)a.n_blocks * a.rows * a.ns;
  for (int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tt < outputs * LS;
       tt += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = tt / LS;
    const int part = (int)(tt - e * LS);
    const int s = (int)(e % a.ns);
    const int64_t t = e / a.ns;
    const int row = (int)(t % a.rows);
    const int blk = (int)(t / a.rows);
    const DBlock b = a.blocks[blk];
    const double* Er = core + ((int64_t)b.unique * a.rows + row) * a.cols;
    T acc[4] = {0, 0, 0, 0};
    int l = part;
    for (; l + 3 * LS < a.cols; l += 4 * LS) {
      T ev[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ev[u] = (T)Er[l + u * LS];
        xv[u] = (T)a.x_in[dense_gather(b, l + u * LS, a.n, a.ndim) * a.ns + s];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(ev[u], xv[u], acc[u]);
    }
    for (; l < a.cols; l += LS)
      acc[0] = fma((T)Er[l], (T)a.x_in[dense_gather(b, l, a.n, a.ndim) * a.ns + s], acc[0]);
    T sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
    for (int off = LS / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (part == 0) {
      const int64_t o = dense_scatter(b, row, a.n, a.ndim) * a.ns + s;
      const double v = (double)sum + (a.bias ? a.bias[o] : 0.0);
      if (!isfinite(v) && a.status) atomicOr(a.status, kStatusNonFinite);
      a.x_out[o] = v;
    }
  }
}

// ------------------------------------------------------ resident steps --
// Small 1D problems with one stored block (a translation-invariant operator
// on cores of `rows` points tiling the grid): every step of a lem_step call
// in one launch.  A workgroup holds the states of `mpw` members in LDS (two
// buffers) and runs all steps: per step Y = E[core,:] X_g, where column
// (block b, member m) of X_g is the box of block b gathered from member m's
// state, on FP64 MFMA (16x16x4).  Wave w owns core rows 16w .. 16w + 15 and
// keeps their stored-block fragments in registers for the whole launch;
// each step is one barrier.  The launch is bound by the MFMA chain of one
// step (cols / 4 products per column tile), not by launch latency.
struct ResidentArgs {
  const double* core;    // rows x cols, row-major
  const double* bias;    // forcing term per step (N x ns) or null
  const double* x_in;
  double* x_out;
  int* status;
  int n, ns, rows, cols, nb, h, n_steps, mpw;
};

constexpr int kResidentMaxCols = 128;  // 32 k-steps of stored-block fragments per lane

// padded LDS index of grid point p: one double after every core, so the 16
// lanes of a fragment read (16 blocks at the same offset) hit distinct banks
__device__ __forceinline__ int resident_pad(int p, int rows) { return p + p / rows; }

template <int NW, int KMAX>
__global__ __launch_bounds__(64 * NW) void dense_resident_kernel(ResidentArgs a) {
  // KMAX k-steps of 4 columns cover the box (columns past it are zero)
  extern __shared__ double xs[];  // [2][mpw][padded n]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int m0 = blockIdx.x * a.mpw, mv = min(a.mpw, a.ns - m0);
  const int pn = a.n + a.n / a.rows + 1;
  double* buf0 = xs;
  double* buf1 = xs + (size_t)a.mpw * pn;
  // this workgroup's members into LDS (members past ns are zero)
  for (int e = tid; e < a.mpw * a.n; e += 64 * NW) {
    const int m = e / a.n, pt = e - m * a.n;
    buf0[m * pn + resident_pad(pt, a.rows)] = m < mv ? a.x_in[(int64_t)pt * a.ns + m0 + m] : 0.0;
  }
  // stored-block fragments of this wave's 16 core rows (zero past the rows
  // and the columns)
  const int row = 16 * w + lr;
  double ek[KMAX];
#pragma unroll
  for (int kk = 0; kk < KMAX; ++kk) {
    const int col = 4 * kk + lk;
    ek[kk] = (row < a.rows && col < a.cols) ? a.core[(int64_t)row * a.cols + col] : 0.0;
  }
  __syncthreads();
  const float inv_rows = 1.0f / (float)a.rows;
  const int ncols = a.nb * a.mpw;          // (block, member) columns, block fastest
  const int ntiles = (ncols + 15) / 16;
  for (int step = 0; step < a.n_steps; ++step) {
    const double* cur = (step & 1) ? buf1 : buf0;
    double* nxt = (step & 1) ? buf0 : buf1;
    for (int t = 0; t < ntiles; ++t) {
      const int q = 16 * t + lr;
      const int b = q % a.nb, m = q / a.nb;
      const bool qv = q < ncols;
      const double* xm = cur + (qv ? m : 0) * pn;
      // box of block b starts h points before its core (periodic); the
      // padded index p + p / rows takes the quotient in single precision,
      // exact here: (p + 1/2) / rows is at least 1 / (2 rows) >= 2^-8 from an
      // integer, above the rounding error of p < 2^14 times a rounded 1/rows
      int p = b * a.rows - a.h + lk;
      p += p < 0 ? a.n : 0;
      // all reads first (always inside the member's state), then the zeros
      // past the box and the columns: a select right after each read would
      // wait for it
      double bv[KMAX];
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk) {
        bv[kk] = xm[p + (int)(((float)p + 0.5f) * inv_rows)];
        p += 4;
        p -= p >= a.n ? a.n : 0;
      }
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk) bv[kk] = (qv && 4 * kk + lk < a.cols) ? bv[kk] : 0.0;
      d4 acc = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ek[kk], bv[kk], acc, 0, 0, 0);
      if (qv) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * w + 4 * i + lk;
          if (r < a.rows) {
            const int pt = b * a.rows + r;
            const double y = acc[i] + (a.bias ? a.bias[(int64_t)pt * a.ns + m0 + m] : 0.0);
            nxt[m * pn + resident_pad(pt, a.rows)] = y;
          }
        }
      }
    }
    __syncthreads();
  }
  const double* fin = (a.n_steps & 1) ? buf1 : buf0;
  bool bad = false;
  for (int e = tid; e < mv * a.n; e += 64 * NW) {
    const int m = e / a.n, pt = e - m * a.n;
    const double y = fin[m * pn + resident_pad(pt, a.rows)];
    bad |= !isfinite(y);
    a.x_out[(int64_t)pt * a.ns + m0 + m] = y;
  }
  latch_nonfinite(bad, a.status);
}

int dense_resident_members(int n, int ns, int rows, int cols, int nb) {
  if (rows < 4 || rows > 128 || cols > kResidentMaxCols || n != nb * rows || cols < 1 ||
      n >= (1 << 14))
    return 0;
  const size_t pn = (size_t)n + n / rows + 1;
  const size_t per = 2 * pn * sizeof(double);  // two buffers of one member
  const size_t lds_max = 160 * 1024;
  if (per > lds_max) return 0;
  // up to 64 (block, member) columns per workgroup, within LDS
  int mpw = std::max(1, 64 / nb);
  mpw = std::min<int>(mpw, (int)(lds_max / per));
  return std::max(1, std::min(mpw, ns));
}

hipError_t dense_resident_steps(const double* core, const double* bias, const double* x_in,
                                double* x_out, int* status, int n, int ns, int rows, int cols,
                                int nb, int h, int n_steps, hipStream_t st) {
  const int mpw = dense_resident_members(n, ns, rows, cols, nb);
  if (mpw < 1 || n_steps < 1 || h < 0 || cols != rows + 2 * h) return hipErrorInvalidValue;
  ResidentArgs a{core, bias, x_in, x_out, status, n, ns, rows, cols, nb, h, n_steps, mpw};
  const size_t lds = 2 * (size_t)mpw * (n + n / rows + 1) * sizeof(double);
  const dim3 g((ns + mpw - 1) / mpw);
  const int nw = (rows + 15) / 16, ks = (cols + 3) / 4;
#define LEM_RES_K(NW_, K_)                                                                 \
  {                                                                                        \
    auto fn = dense_resident_kernel<NW_, K_>;                                              \
    if (lds > 64 * 1024) {                                                                 \
      hipError_t e = hipFuncSetAttribute((const void*)fn,                                  \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e != hipSuccess) return e;                                                       \
    }                                                                                      \
    hipLaunchKernelGGL(fn, g, dim3(64 * NW_), lds, st, a);                                 \
  }
#define LEM_RES(NW_)                                                                       \
  if (ks <= 8) LEM_RES_K(NW_, 8)                                                           \
  else if (ks <= 16) LEM_RES_K(NW_, 16)                                                    \
  else if (ks <= 24) LEM_RES_K(NW_, 24)                                                    \
  else LEM_RES_K(NW_, 32)
  switch (nw) {
    case 1: LEM_RES(1) break;
    case 2: LEM_RES(2) break;
    case 3: LEM_RES(3) break;
    case 4: LEM_RES(4) break;
    case 5: LEM_RES(5) break;
    case 6: LEM_RES(6) break;
    case 7: LEM_RES(7) break;
    default: LEM_RES(8) break;
  }
#undef LEM_RES
#undef LEM_RES_K
  return hipGetLastError();
}

// -------------------------------------------------------------- launchers --

static inline dim3 grid1(int64_t total, int per = 256, int cap = 8192) {
  int64_t g = (total + per - 1) / per;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

hipError_t dense_assemble(const void* ops, double* A, int nl, int nu, hipStream_t st) {
  dim3 g = grid1((int64_t)nl * nl);
  g.y = nu;
  hipLaunchKernelGGL(assemble_kernel, g, dim3(256), 0, st, (const DenseOp*)ops, A, nl);
  return hipGetLastError();
}

// Local matrices of a variable-coefficient operator (face diffusion numbers
// mux, muy and, with face velocities, ax, ay, all dt-scaled): dt*A_M of every
// box in [u0, u0 + count), one workgroup per row.  The row weights are those
// of the conservative form (section 4.3), couplings leaving the box dropped.
struct VarOp {
  const double* mux;
  const double* muy;
  const double* ax;  // null: constant velocity (chx, chy)
  const double* ay;
  double chx, chy;
  int n, ndim;
};

struct VarBox {
  int ox, oy, h, Lx, Ly;
};

__global__ void var_assemble_kernel(VarOp o, const VarBox* boxes, int nl, double* A) {
  const int u = blockIdx.y, r = blockIdx.x;
  const VarBox b = boxes[u];
  const int n = o.n;
  const int ry = r / b.Lx, rx = r - ry * b.Lx;
  const int gx = wrap(b.ox - b.h + rx, n);
  const int gy = o.ndim == 2 ? wrap(b.oy - b.h + ry, n) : 0;
  const int64_t g = (int64_t)gy * n + gx, gw = (int64_t)gy * n + wrap(gx - 1, n);
  const double me = o.mux[g], mw = o.mux[gw];
  double mn = 0.0, ms = 0.0, an = 0.0, as = 0.0;
  const int64_t gs = (int64_t)wrap(gy - 1, n) * n + gx;
  if (o.ndim == 2) { mn = o.muy[g]; ms = o.muy[gs]; }
  double w0 = -(me + mw + mn + ms), wW, wE, wS = 0.0, wN = 0.0;
  if (o.ax) {
    const double ae = o.ax[g], aw = o.ax[gw];
    if (o.ndim == 2) { an = o.ay[g]; as = o.ay[gs]; }
    w0 -= (ae - aw) + (an - as);
    wW = mw + aw;
    wE = me - ae;
    if (o.ndim == 2) { wS = ms + as; wN = mn - an; }
  } else {
    wW = mw + o.chx;
    wE = me - o.chx;
    if (o.ndim == 2) { wS = ms + o.chy; wN = mn - o.chy; }
  }
  double* row = A + ((int64_t)u * nl + r) * nl;
  for (int c = threadIdx.x; c < nl; c += blockDim.x) {
    double v = 0.0;
    if (c == r) v = w0;
    else if (c == r - 1 && rx > 0) v = wW;
    else if (c == r + 1 && rx < b.Lx - 1) v = wE;
    else if (c == r - b.Lx && ry > 0) v = wS;
    else if (c == r + b.Lx && ry < b.Ly - 1) v = wN;
    row[c] = v;
  }
}

size_t dense_varbox_size() { return sizeof(VarBox); }

void dense_varbox_fill(void* dst, int i, int ox, int oy, int h, int Lx, int Ly) {
  VarBox* b = (VarBox*)dst + i;
  b->ox = ox; b->oy = oy; b->h = h; b->Lx = Lx; b->Ly = Ly;
}

hipError_t dense_assemble_var(const double* mux, const double* muy, const double* ax,
                              const double* ay, double chx, double chy, int n, int ndim,
                              const void* boxes, int count, int nl, double* A, hipStream_t st) {
  VarOp o{mux, muy, ax, ay, chx, chy, n, ndim};
  hipLaunchKernelGGL(var_assemble_kernel, dim3((unsigned)nl, (unsigned)count), dim3(256), 0, st,
                     o, (const VarBox*)boxes, nl, A);
  return hipGetLastError();
}

// [[dt A_M, I], [0, 0]] (size 2 nl): its exponential holds phi_1(dt A_M) in
// the top-right block (the forcing term of update (5)).
__global__ void assemble_aug_kernel(const DenseOp* ops, double* A, int nl) {
  const int u = blockIdx.y;
  const DenseOp o = ops[u];
  const int n2 = 2 * nl;
  double* M = A + (int64_t)u * n2 * n2;
  const int64_t total = (int64_t)n2 * n2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n2), c = (int)(e - (int64_t)r * n2);
    double v = 0.0;
    if (r < nl && c >= nl) {
      v = (c - nl == r) ? 1.0 : 0.0;
    } else if (r < nl) {
      const int ry = r / o.Lx, rx = r - ry * o.Lx;
      if (c == r) v = o.w0;
      else if (c == r - 1 && rx > 0) v = o.wW;
      else if (c == r + 1 && rx < o.Lx - 1) v = o.wE;
      else if (c == r - o.Lx && ry > 0) v = o.wS;
      else if (c == r + o.Lx && ry < o.Ly - 1) v = o.wN;
    }
    M[e] = v;
  }
}

hipError_t dense_assemble_aug(const void* ops, double* A, int nl, int nu, hipStream_t st) {
  dim3 g = grid1((int64_t)4 * nl * nl);
  g.y = nu;
  hipLaunchKernelGGL(assemble_aug_kernel, g, dim3(256), 0, st, (const DenseOp*)ops, A, nl);
  return hipGetLastError();
}

size_t dense_op_size() { return sizeof(DenseOp); }

void dense_op_fill(void* dst, int i, double w0, double wW, double wE, double wS,
                   double wN, int Lx, int Ly) {
  DenseOp* o = (DenseOp*)dst + i;
  o->w0 = w0; o->wW = wW; o->wE = wE; o->wS = wS; o->wN = wN; o->Lx = Lx; o->Ly = Ly;
}

hipError_t dense_norm1(const double* A, int nl, int nu, double* norms, hipStream_t st) {
  hipLaunchKernelGGL(norm1_kernel, dim3(nu), dim3(256), 0, st, A, nl, norms);
  return hipGetLastError();
}

hipError_t dense_scale_pow2(double* A, int nl, int nu, const int* s, hipStream_t st) {
  dim3 g = grid1((int64_t)nl * nl);
  g.y = nu;
  hipLaunchKernelGGL(scale_pow2_kernel, g, dim3(256), 0, st, A, nl, s);
  return hipGetLastError();
}

hipError_t dense_gemm(const double* A, const double* B, double* C, int nl, int nu,
                      hipStream_t st) {
  const int t = (nl + 63) / 64;
  hipLaunchKernelGGL(dgemm_kernel, dim3(t, t, nu), dim3(256), 0, st, A, B, C, nl,
                     (int64_t)nl * nl);
  return hipGetLastError();
}

hipError_t dense_lincomb(const double* X0, double c0, const double* X1, double c1,
                         const double* X2, double c2, const double* X3, double c3,
                         double d, double* out, int nl, int nu, hipStream_t st) {
  LinComb p;
  p.X[0] = X0; p.X[1] = X1; p.X[2] = X2; p.X[3] = X3;
  p.c[0] = c0; p.c[1] = c1; p.c[2] = c2; p.c[3] = c3;
  p.d = d; p.out = out; p.nl = nl; p.stride = (int64_t)nl * nl;
  dim3 g = grid1((int64_t)nl * nl);
  g.y = nu;
  hipLaunchKernelGGL(lincomb_kernel, g, dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t dense_pade_pq(double* V, double* U, int64_t total, hipStream_t st) {
  hipLaunchKernelGGL(pade_pq_kernel, grid1(total), dim3(256), 0, st, V, U, total);
  return hipGetLastError();
}

hipError_t dense_solve(double* Q, double* P, int nl, int nu, hipStream_t st) {
  const int64_t stride = (int64_t)nl * nl;
  for (int j = 0; j < nl; ++j) {
    hipLaunchKernelGGL(lu_pivot_kernel, dim3(nu), dim3(256), 0, st, Q, P, nl, stride, j);
    const int rows = nl - j - 1;
    if (rows > 0) {
      const int cols = (nl - j - 1) + nl;
      hipLaunchKernelGGL(lu_elim_kernel, dim3((cols + 255) / 256, rows, nu), dim3(256), 0, st,
                         Q, P, nl, stride, j);
    }
  }
  for (int j = nl - 1; j > 0; --j)
    hipLaunchKernelGGL(lu_back_kernel, dim3((nl + 255) / 256, j, nu), dim3(256), 0, st, Q, P,
                       nl, stride, j);
  hipLaunchKernelGGL(lu_diag_kernel, dim3((nl + 255) / 256, nl, nu), dim3(256), 0, st, Q, P,
                     nl, stride);
  return hipGetLastError();
}

hipError_t dense_pack(const double* R, int nl, int Lx, int h, int cx, int cy, int ndim,
                      int rows, int rows_p, int cols_p, double* e64, float* e32,
                      void* e16, double* core_out, hipStream_t st) {
  PackArgs a{R, nl, Lx, h, cx, cy, ndim, rows, rows_p, cols_p, e64, e32,
             (__hip_bfloat16*)e16, core_out};
  hipLaunchKernelGGL(pack_kernel, grid1((int64_t)rows_p * cols_p), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t dense_block_size() { return sizeof(DBlock); }

void dense_block_fill(void* dst, int i, int ox, int oy, int cx, int cy, int h, int Lx,
                      int Ly, int unique) {
  DBlock* d = (DBlock*)dst + i;
  d->ox = ox; d->oy = oy; d->cx = cx; d->cy = cy; d->h = h; d->Lx = Lx; d->Ly = Ly;
  d->unique = unique;
}

// tile shapes of the FP64/FP32 apply (rows per wave, K chunk, waves per workgroup)
static const int kApplyShapes[kApplyConfigs][3] = {{32, 16, 4}, {32, 32, 4}, {32, 32, 8},
                                                   {64, 32, 4}, {16, 32, 8}, {16, 32, 4},
                                                   {16, 16, 8}, {16, 32, 16}};

bool dense_apply_supported(int precision, int cfg, int ns, int rows_p, int cols_p,
                           int64_t n_points) {
  if (ns % 64 != 0) return precision == 0 || precision == 1;  // small-ensemble kernel
  if (precision == 0 || precision == 1) {
    if (cfg < 0 || cfg >= kApplyConfigs) return false;
    // a live wave reads wm rows of E: the padded rows must be a multiple of wm
    return rows_p % kApplyShapes[cfg][0] == 0 && cols_p % kApplyShapes[cfg][1] == 0;
  }
  if (precision != 2 && precision != 3) return false;
  if (cfg < 0 || cfg >= kApplyBf16Configs) return false;
  if (cfg == 4)  // 128 states per workgroup, 32-bit grid points in LDS
    return ns % 128 == 0 && rows_p % 32 == 0 && cols_p % 32 == 0 &&
           n_points < ((int64_t)1 << 31) && (size_t)cols_p * sizeof(int) <= 64 * 1024;
  const int wm = (cfg & 1) ? 64 : 32;
  return rows_p % wm == 0 && cols_p % 32 == 0 && (size_t)cols_p * sizeof(int64_t) <= 64 * 1024;
}

hipError_t dense_apply(int precision, int cfg, const void* blocks, const void* E,
                       int64_t e_stride, const double* core, const double* x_in,
                       double* x_out, int n, int ndim, int ns, int rows, int rows_p,
                       int cols, int cols_p, int n_blocks, const double* bias, int* status,
                       hipStream_t st, const void* xpieces, int64_t n_points) {
  ApplyArgs a;
  a.bias = bias;
  a.status = status;
  a.xp = nullptr;
  a.blocks = (const DBlock*)blocks; a.E = E; a.e_stride = e_stride;
  a.x_in = x_in; a.x_out = x_out; a.n = n; a.ndim = ndim; a.ns = ns;
  a.rows = rows; a.rows_p = rows_p; a.cols = cols; a.cols_p = cols_p;
  a.n_blocks = n_blocks;
  if (ns % 64 != 0) {
    a.row_tiles = 1; a.col_tiles = 1;
    const dim3 g = grid1((int64_t)n_blocks * rows * ns * 8, 256, 65535);  // 8 lanes per output
    if (precision == 0)
      hipLaunchKernelGGL(apply_simple_kernel<double>, g, dim3(256), 0, st, a, core);
    else if (precision == 1)
      hipLaunchKernelGGL(apply_simple_kernel<float>, g, dim3(256), 0, st, a, core);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  a.col_tiles = ns / 64;
  if (!dense_apply_supported(precision, cfg, ns, rows_p, cols_p, n_points))
    return hipErrorInvalidValue;
  if (precision == 0 || precision == 1) {
    const int wm = kApplyShapes[cfg][0], nw = kApplyShapes[cfg][2];
    a.row_tiles = (rows_p + nw * wm - 1) / (nw * wm);
    const dim3 g(n_blocks * a.row_tiles * a.col_tiles), blk(64 * nw);
#define LEM_APPLY(T)                                                                         \
    switch (cfg) {                                                                           \
      case 0: hipLaunchKernelGGL((apply_mfma_kernel<T, 32, 16, 4>), g, blk, 0, st, a); break; \
      case 1: hipLaunchKernelGGL((apply_mfma_kernel<T, 32, 32, 4>), g, blk, 0, st, a); break; \
      case 2: hipLaunchKernelGGL((apply_mfma_kernel<T, 32, 32, 8>), g, blk, 0, st, a); break; \
      case 3: hipLaunchKernelGGL((apply_mfma_kernel<T, 64, 32, 4>), g, blk, 0, st, a); break; \
      case 4: hipLaunchKernelGGL((apply_mfma_kernel<T, 16, 32, 8>), g, blk, 0, st, a); break; \
      case 5: hipLaunchKernelGGL((apply_mfma_kernel<T, 16, 32, 4>), g, blk, 0, st, a); break; \
      case 6: hipLaunchKernelGGL((apply_mfma_kernel<T, 16, 16, 8>), g, blk, 0, st, a); break; \
      default: hipLaunchKernelGGL((apply_mfma_kernel<T, 16, 32, 16>), g, blk, 0, st, a); break; \
    }
    if (precision == 0) { LEM_APPLY(double) } else { LEM_APPLY(float) }
#undef LEM_APPLY
    return hipGetLastError();
  }
  // split-bf16 shapes: rows per wave 32 (ids 0, 2, 4) or 64 (1, 3), four
  // waves (ids 0, 1) or eight (2, 3, 4) per workgroup, 64 states per
  // workgroup or 128 (id 4)
  const int wm = (cfg == 1 || cfg == 3) ? 64 : 32, nw = cfg >= 2 ? 8 : 4;
  const int bn = cfg == 4 ? 128 : 64;
  a.col_tiles = ns / bn;
  a.row_tiles = (rows_p + nw * wm - 1) / (nw * wm);
  const dim3 g(n_blocks * a.row_tiles * a.col_tiles);
  // gathered row offsets (dynamic LDS beside the static X stages)
  const size_t gl = (size_t)cols_p * (bn == 128 ? sizeof(int) : sizeof(int64_t));
  if (xpieces) a.xp = (const __bf16*)xpieces;  // split by dense_split_pieces
#define LEM_BF16(NT_, WM_, NW_, BN_)                                                       \
  {                                                                                        \
    auto fn = a.xp ? apply_bf16_kernel<NT_, WM_, NW_, true, BN_>                           \
                   : apply_bf16_kernel<NT_, WM_, NW_, false, BN_>;                         \
    if (BN_ == 128) {                                                                      \
      hipError_t e = hipFuncSetAttribute((const void*)fn,                                  \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)gl); \
      if (e != hipSuccess) return e;                                                       \
    }                                                                                      \
    hipLaunchKernelGGL(fn, g, dim3(64 * NW_), gl, st, a);                                  \
  }
#define LEM_BF16_SHAPES(NT_)                              \
  switch (cfg) {                                          \
    case 0: LEM_BF16(NT_, 32, 4, 64) break;               \
    case 1: LEM_BF16(NT_, 64, 4, 64) break;               \
    case 2: LEM_BF16(NT_, 32, 8, 64) break;               \
    case 3: LEM_BF16(NT_, 64, 8, 64) break;               \
    default: LEM_BF16(NT_, 32, 8, 128) break;             \
  }
  if (precision == 2) {
    LEM_BF16_SHAPES(3)
  } else if (precision == 3) {
    LEM_BF16_SHAPES(6)
  } else {
    return hipErrorInvalidValue;
  }
#undef LEM_BF16_SHAPES
#undef LEM_BF16
  return hipGetLastError();
}

hipError_t dense_split_pieces(const double* x, int64_t total, int np, void* pieces,
                              hipStream_t st) {
  if (np == 2)
    hipLaunchKernelGGL(split_pieces_kernel<2>, grid1(total), dim3(256), 0, st, x, total,
                       (bf16x2*)pieces);
  else if (np == 3)
    hipLaunchKernelGGL(split_pieces_kernel<3>, grid1(total), dim3(256), 0, st, x, total,
                       (bf16x4*)pieces);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace lem
