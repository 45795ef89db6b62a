// Device-side building blocks shared by the LEM kernels (gfx950, wave64).
//
//  * KBlock: self-contained descriptor of one region M_i = D_i u B_i of the
//    overlapping decomposition (section 3): core box, buffer width, stencil
//    weights of dt_sub*A, Krylov dimension and sub-step count, and where its
//    state lives.  Kernels compute the gather index of every local point and
//    the scatter index of every core point from the box alone, so no index
//    map is read on the hot path.
//  * Workgroup reductions built from wave64 cross-lane sums.
//  * expm_small: Pade [13/13] scaling and squaring (Higham 2005) of a small
//    dense matrix held in LDS, computed cooperatively by one workgroup in
//    float64; used for the Krylov projections exp(H_m).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lem {

constexpr int kMaxKrylov = 48;  // largest Krylov dimension handled on device

// Status bits latched by kernels (combined with atomicOr).
constexpr int kStatusNotConverged = 1;
constexpr int kStatusNonFinite = 2;

struct KBlock {
  double w0, wW, wE, wS, wN;  // constant weights of dt_sub*A (mu_off < 0)
  double chx, chy;            // dt_sub * C_x / 2, dt_sub * C_y / 2 (variable nu)
  double sub_scale;           // 1 / nsub: scales dt-based face mu's to dt_sub
  double tol;                 // relative tolerance of the Krylov estimate
  int64_t x_off;              // first double of this problem's state array
  int64_t mu_off;             // face-mu arrays (mux then muy, N each); -1 = const
  int64_t v_off;              // basis work offset in doubles (global-basis form)
  int32_t n, ndim;            // grid side and dimension of this problem
  int32_t ox, oy, cx, cy, h;  // core origin and size, buffer width
  int32_t Lx, Ly;             // local box = (cx + 2h) x (cy + 2h)   (Ly = 1 in 1D)
  int32_t m, nsub;            // Krylov dimension, equal sub-steps per step
  int32_t ns;                 // ensemble size (stride of the state arrays)
  int32_t diag;               // index of this block's estimate slot
  int32_t periodic;           // bit 0 (1): the core spans the whole x axis,
                              // bit 1 (2): the whole y axis; the box keeps the
                              // periodic coupling along such an axis and has
                              // no buffer across it (D = 1: both bits)
  int32_t aug;                // 1: forced step, the box carries one extra
                              // (augmented) coordinate after its Lx*Ly points
  int32_t hy;                 // buffer width along y (h is the one along x)
  int32_t varvel;             // 1: face velocities follow the face mu's in the
                              // coefficient arrays (ax at mu_off + 2N, ay at
                              // mu_off + 3N; conservative centered advection)
  int32_t stage;              // 1: the kernel stages the face mu's of the box
                              // in LDS (set when the launch reserves the room)
  double gscale;              // dt_sub: scales the forcing to the sub-step
  const double* force;        // forcing g (rate units), N x ns, or null
  // Optional per-block buffers (null: the launch's arguments).  A serving
  // launch mixes blocks of independent problems, each with its own state,
  // coefficients and basis work space.
  const double* xin;
  double* xout;
  const double* coef;
  double* vwork;
  int* status;                // status word of this block's problem, or null
  // Large-box kernel: the five stencil weights of dt_sub A_M per box point,
  // precomputed once per block (shared by its members): weight k of local
  // point l at wts[k * NT * P + l] for the launch shape (NT, P); null: the
  // kernel computes them from the coefficients on every use.
  const double* wts;
};

// One region of the Kronecker-factored dense method: a c x c core with an
// h-point buffer (box side L = c + 2h) of a 2D constant-coefficient operator
// on an n x n grid, and the core rows of the two 1D local exponentials.
struct KronBlock {
  int32_t ox, oy, c, h, L, n, ns, pad;
  const double* x_in;   // state of this block's problem (N x ns)
  double* x_out;
  const double* ex;     // c x L: rows h..h+c-1 of exp(dt A_x) on the box
  const double* ey;     // c x L: rows h..h+c-1 of exp(dt A_y)
  int* status;          // status word of this block's problem, or null
};

struct KrylovArgs {
  const KBlock* blocks;
  const double* x_in;
  double* x_out;
  const double* coef;   // face-mu arrays of variable-coefficient problems
  double* vwork;        // global-basis work space
  double* diag;         // per (block, state) relative estimate of the step
  int* status;          // latched status bits
  double* calib;        // calibration output (mode 1)
  int mode;             // 0: step; 1: calibrate (Arnoldi only, write H)
  int n_blocks;
};

__device__ __forceinline__ int wrap(int a, int n) {
  // callers are almost always within one period of the range: no division
  if (a >= 0 && a < n) return a;
  if (a < 0 && a >= -n) return a + n;
  if (a >= n && a < 2 * n) return a - n;
  a %= n;
  return a < 0 ? a + n : a;
}

// Global DOF of local point (lx, ly) of block b.
__device__ __forceinline__ int64_t gather_index(const KBlock& b, int lx, int ly) {
  const int gx = wrap(b.ox - b.h + lx, b.n);
  if (b.ndim == 1) return gx;
  const int gy = wrap(b.oy - b.hy + ly, b.n);
  return (int64_t)gy * b.n + gx;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Butterfly reduce-scatter over the wave: K values per lane in, the wave
// total of value (lane >> log2(64/K)) out.
template <int K>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[K]) {
  const int lane = threadIdx.x & 63;
  int c = K;
#pragma unroll
  for (int o = 32; o >= 64 / K; o >>= 1) {
    const int half = c >> 1;
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
      if (i < half) {
        double lo = v[i], hi = v[i + half];
        // keep the selects on register values: folded into an indexed load of
        // v they would demote the whole array to scratch memory
        asm volatile("" : "+v"(lo), "+v"(hi));
        const double send = upper ? lo : hi;
        const double keep = upper ? hi : lo;
        v[i] = keep + __shfl_xor(send, o, 64);
      }
    }
    c = half;
  }
  double r = v[0];
#pragma unroll
  for (int o = 32 / K; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
  return r;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sums K per-thread values over the workgroup; thread-uniform `cnt` <= K of
// them are live.  Results land in out[0..cnt) (LDS), visible to every thread
// on return.  red must hold (NT/64)*K doubles.
template <int NT, int K>
__device__ __forceinline__ void wg_sum(double (&v)[K], int cnt, double* red,
                                       double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q)
    if (q < cnt) v[q] = wave_sum(v[q]);
  if (NT == 64) {
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (q < cnt) out[q] = v[q];
    }
    __syncthreads();
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q)
      if (q < cnt) red[wv * K + q] = v[q];
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * K + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double wg_sum1(double v, double* red) {
  double a[1] = {v};
  wg_sum<NT, 1>(a, 1, red, red + NT / 64);
  const double r = red[NT / 64];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Small dense matrix exponential in LDS.
// ---------------------------------------------------------------------------

// Pade [13/13] numerator coefficients b_0..b_13 (Higham 2005, scaled b_13 = 1)
// and the scaling threshold theta_13 of the same paper.
__device__ constexpr double kPadeB[14] = {
    64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
    1187353796428800.0,  129060195264000.0,   10559470521600.0,
    670442572800.0,      33522128640.0,       1323241920.0,
    40840800.0,          960960.0,            16380.0,
    182.0,               1.0};
constexpr double kTheta13 = 5.371920351148152;

// C = A * B for m x m row-major matrices in LDS (leading dimension m).
template <int NT>
__device__ __forceinline__ void lds_matmul(const double* A, const double* B,
                                           double* C, int m) {
  const int mm = m * m;
  for (int idx = threadIdx.x; idx < mm; idx += NT) {
    const int i = idx / m, j = idx - i * m;
    const double* a = A + i * m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s = fma(a[k], B[k * m + j], s);
    C[idx] = s;
  }
  __syncthreads();
}

// R = exp(A) for the m x m matrix A (LDS, row-major, destroyed); inlined into
// each kernel (one out-of-line copy shared by two kernels of different LDS
// layouts is rejected by the gfx950 backend).  W holds
// 5*m*m doubles of LDS work space, piv at least 2*NT/64 + 4 doubles.  Every
// thread of the workgroup must call it; R is visible to all on return.
template <int NT>
__device__ __forceinline__ void expm_small(double* A, int m, double* W, double* R, double* piv) {
  const int tid = threadIdx.x;
  const int mm = m * m;
  double* A2 = W;
  double* A4 = W + mm;
  double* A6 = W + 2 * mm;
  double* U = W + 3 * mm;
  double* V = W + 4 * mm;
  // 1-norm -> number of squarings s
  double cs = 0.0;
  for (int j = tid; j < m; j += NT) {
    double t = 0.0;
    for (int i = 0; i < m; ++i) t += fabs(A[i * m + j]);
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
  if (cs > kTheta13 && cs < 1e300) s = min(60, (int)ceil(log2(cs / kTheta13)));
  if (s > 0) {
    for (int idx = tid; idx < mm; idx += NT) A[idx] = ldexp(A[idx], -s);
    __syncthreads();
  }
  const double* b = kPadeB;
  lds_matmul<NT>(A, A, A2, m);
  lds_matmul<NT>(A2, A2, A4, m);
  lds_matmul<NT>(A4, A2, A6, m);
  // U = A (A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I)
  for (int idx = tid; idx < mm; idx += NT)
    V[idx] = b[13] * A6[idx] + b[11] * A4[idx] + b[9] * A2[idx];
  __syncthreads();
  lds_matmul<NT>(A6, V, U, m);
  for (int idx = tid; idx < mm; idx += NT) {
    const int i = idx / m, j = idx - i * m;
    U[idx] += b[7] * A6[idx] + b[5] * A4[idx] + b[3] * A2[idx] + (i == j ? b[1] : 0.0);
  }
  __syncthreads();
  lds_matmul<NT>(A, U, R, m);  // R holds U for now
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  for (int idx = tid; idx < mm; idx += NT)
    U[idx] = b[12] * A6[idx] + b[10] * A4[idx] + b[8] * A2[idx];
  __syncthreads();
  lds_matmul<NT>(A6, U, V, m);
  for (int idx = tid; idx < mm; idx += NT) {
    const int i = idx / m, j = idx - i * m;
    const double v = V[idx] + b[6] * A6[idx] + b[4] * A4[idx] + b[2] * A2[idx] +
                     (i == j ? b[0] : 0.0);
    const double u = R[idx];
    V[idx] = v + u;  // P = V + U (right-hand sides)
    U[idx] = v - u;  // Q = V - U
  }
  __syncthreads();
  // Solve Q X = P by Gaussian elimination with partial pivoting on [Q | P].
  double* Q = U;
  double* P = V;
  double* fac = A;  // reuse A's storage for the column multipliers
  for (int j = 0; j < m; ++j) {
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int i = j + tid; i < m; i += 64) {
        const double a = fabs(Q[i * m + j]);
        if (a > best) { best = a; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) piv[0] = (double)bi;
    }
    __syncthreads();
    const int p = (int)piv[0];
    if (p != j) {
      for (int k = tid; k < 2 * m; k += NT) {
        double* M = k < m ? Q : P;
        const int kk = k < m ? k : k - m;
        const double t = M[j * m + kk];
        M[j * m + kk] = M[p * m + kk];
        M[p * m + kk] = t;
      }
      __syncthreads();
    }
    const double inv = 1.0 / Q[j * m + j];
    for (int i = j + 1 + tid; i < m; i += NT) fac[i] = Q[i * m + j] * inv;
    __syncthreads();
    const int rows = m - j - 1;
    const int cols = (m - j - 1) + m;  // trailing Q columns, then all of P
    for (int idx = tid; idx < rows * cols; idx += NT) {
      const int r = j + 1 + idx / cols;
      const int c = idx % cols;
      if (c < m - j - 1) {
        const int k = j + 1 + c;
        Q[r * m + k] = fma(-fac[r], Q[j * m + k], Q[r * m + k]);
      } else {
        const int k = c - (m - j - 1);
        P[r * m + k] = fma(-fac[r], P[j * m + k], P[r * m + k]);
      }
    }
    __syncthreads();
  }
  // Back substitution: rows of X overwrite rows of P from the bottom up.
  for (int j = m - 1; j >= 0; --j) {
    const double inv = 1.0 / Q[j * m + j];
    for (int k = tid; k < m; k += NT) P[j * m + k] *= inv;
    __syncthreads();
    for (int idx = tid; idx < j * m; idx += NT) {
      const int r = idx / m, k = idx - r * m;
      P[r * m + k] = fma(-Q[r * m + j], P[j * m + k], P[r * m + k]);
    }
    __syncthreads();
  }
  // Square s times.
  double* src = P;
  double* dst = A2;
  for (int q = 0; q < s; ++q) {
    lds_matmul<NT>(src, src, dst, m);
    double* t = src; src = dst; dst = t;
  }
  for (int idx = tid; idx < mm; idx += NT) R[idx] = src[idx];
  __syncthreads();
}

}  // namespace lem
