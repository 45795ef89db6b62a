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

// y(core) = x(core) + sum_l Phi[blk][row][l][s] f(gather(l), s): one thread
// per (block, core row, member), consecutive threads on consecutive members.
__global__ void ere_apply_kernel(const double* __restrict__ x, const double* __restrict__ f,
                                 const double* __restrict__ Phi, const EreBox* boxes, int nb,
                                 int ns, int nl, int rows, int n, double* y) {
  const int64_t total = (int64_t)nb * rows * ns;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e % ns);
    const int64_t t = e / ns;
    const int row = (int)(t % rows);
    const int blk = (int)(t / rows);
    const EreBox b = boxes[blk];
    const double* ph = Phi + (t * nl) * ns + s;
    double acc = 0.0;
    for (int l = 0; l < nl; ++l)
      acc = fma(ph[(int64_t)l * ns], f[(int64_t)ere_wrap(b.ox - b.h + l, n) * ns + s], acc);
    const int64_t o = (int64_t)(b.ox + row) * ns + s;
    y[o] = x[o] + acc;
  }
}

// phi_1(dt J_M) for boxes of nl <= 80 points, one workgroup per (block,
// member), everything in LDS: W = dt J_M / 2^s with |W|_1 <= 1/2, F = phi_1(W)
// by its Taylor polynomial of degree 16 (Horner), E = e^W = I + W F, then s
// doublings phi_1(2W) = phi_1(W)(e^W + I)/2, e^{2W} = (e^W)^2.  Products on
// FP64 MFMA (16x16x4) over 16-padded tiles (row stride mp + 1 against LDS
// bank conflicts); each product is formed in registers before it overwrites
// its operand.  Writes the core rows of F into Phi[blk][row][l][s] and the
// number of doublings into sq_out[blk * ns + s].
typedef double d4e __attribute__((ext_vector_type(4)));
constexpr int kPhiMaxN = 80;   // LDS: three 80x80 float64 matrices
constexpr int kPhiTiles = 7;   // output tiles per wave (25 tiles, 4 waves)

template <int NT>
__device__ __forceinline__ void tiles_product(const double* A, const double* B, int mp, int ld,
                                              d4e (&acc)[kPhiTiles]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nt = mp / 16, tiles = nt * nt;
#pragma unroll
  for (int q = 0; q < kPhiTiles; ++q) {
    acc[q] = (d4e){0.0, 0.0, 0.0, 0.0};
    const int t = wv + q * (NT / 64);
    if (t < tiles) {
      const int ti = t / nt, tj = t - ti * nt;
      for (int k0 = 0; k0 < mp; k0 += 4) {
        const double a = A[(ti * 16 + (lane & 15)) * ld + k0 + (lane >> 4)];
        const double b = B[(k0 + (lane >> 4)) * ld + tj * 16 + (lane & 15)];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
  }
}

// C(i, j) = f(i, j, product(i, j)) for this thread's product entries
template <int NT, typename Fn>
__device__ __forceinline__ void tiles_store(const d4e (&acc)[kPhiTiles], int mp, Fn f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nt = mp / 16, tiles = nt * nt;
#pragma unroll
  for (int q = 0; q < kPhiTiles; ++q) {
    const int t = wv + q * (NT / 64);
    if (t < tiles) {
      const int ti = t / nt, tj = t - ti * nt;
#pragma unroll
      for (int r = 0; r < 4; ++r) f(ti * 16 + 4 * r + (lane >> 4), tj * 16 + (lane & 15), acc[q][r]);
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void ere_phi1_kernel(const double* __restrict__ x,
                                                      const EreBox* boxes, int ns, int nl,
                                                      int rows, int n, double dt, double dx,
                                                      double nu, double* Phi, int* sq_out,
                                                      int* status) {
  extern __shared__ double sm[];
  const int mp = (nl + 15) / 16 * 16, mm = mp * mp, ld = mp + 1, ms = mp * ld;
  double* W = sm;
  double* F = sm + ms;
  double* E = sm + 2 * ms;
  double* red = sm + 3 * ms;  // NT/64 partial maxima
  const int tid = threadIdx.x;
  const int blk = blockIdx.x / ns, s = blockIdx.x - blk * ns;
  const EreBox b = boxes[blk];
  const double d = nu / (dx * dx), a = 1.0 / (2.0 * dx);
  // W = dt J_M (zero padding)
  for (int e = tid; e < mm; e += NT) {
    const int r = e / mp, c = e - r * mp;
    double v = 0.0;
    if (r < nl && c < nl) {
      const int lm = r > 0 ? r - 1 : (b.whole ? nl - 1 : -1);
      const int lp = r < nl - 1 ? r + 1 : (b.whole ? 0 : -1);
      if (c == r) v = -2.0 * d;
      else if (c == lm) v = x[(int64_t)ere_wrap(b.ox - b.h + lm, n) * ns + s] * a + d;
      else if (c == lp) v = -x[(int64_t)ere_wrap(b.ox - b.h + lp, n) * ns + s] * a + d;
      v *= dt;
    }
    W[r * ld + c] = v;
  }
  __syncthreads();
  // s = ceil(log2(|W|_1 / 0.5))
  double cs = 0.0;
  for (int c = tid; c < mp; c += NT) {
    double t = 0.0;
    for (int r = 0; r < mp; ++r) t += fabs(W[r * ld + c]);
    cs = fmax(cs, t);
  }
  for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = cs;
  __syncthreads();
  double nrm = 0.0;
  for (int w = 0; w < NT / 64; ++w) nrm = fmax(nrm, red[w]);
  int sq = 0;
  if (nrm > 0.5 && nrm < 1e300) sq = min(40, (int)ceil(log2(nrm / 0.5)));
  if (tid == 0) {
    sq_out[blockIdx.x] = sq;
    if (!(nrm < 1e300)) atomicOr(status, kStatusNonFinite);
  }
  const double scale = ldexp(1.0, -sq);
  for (int e = tid; e < mm; e += NT) {
    const int r = e / mp, c = e - r * mp;
    W[r * ld + c] *= scale;
    // Horner start: F = I / 17!
    F[r * ld + c] = (r == c) ? 2.8114572543455207632e-15 : 0.0;
  }
  __syncthreads();
  // F <- W F + I/(k+1)!  for k = 15 .. 0  (1/(k+1)! by repeated division)
  double inv_fact = 2.8114572543455207632e-15 * 17.0;  // 1/16!
  d4e acc[kPhiTiles];
  for (int k = 15; k >= 0; --k) {
    tiles_product<NT>(W, F, mp, ld, acc);
    __syncthreads();
    const double cdiag = inv_fact;  // 1/(k+1)!
    tiles_store<NT>(acc, mp, [&](int i, int j, double v) { F[i * ld + j] = v + (i == j ? cdiag : 0.0); });
    __syncthreads();
    inv_fact *= (double)(k + 1);
  }
  // E = I + W F
  tiles_product<NT>(W, F, mp, ld, acc);
  tiles_store<NT>(acc, mp, [&](int i, int j, double v) { E[i * ld + j] = v + (i == j ? 1.0 : 0.0); });
  __syncthreads();
  // doublings
  for (int q = 0; q < sq; ++q) {
    tiles_product<NT>(F, E, mp, ld, acc);  // F e^W
    __syncthreads();
    tiles_store<NT>(acc, mp, [&](int i, int j, double v) { F[i * ld + j] = 0.5 * (v + F[i * ld + j]); });
    __syncthreads();
    tiles_product<NT>(E, E, mp, ld, acc);
    __syncthreads();
    tiles_store<NT>(acc, mp, [&](int i, int j, double v) { E[i * ld + j] = v; });
    __syncthreads();
  }
  // core rows of F
  const int64_t base = (int64_t)blk * rows * nl * ns;
  for (int e = tid; e < rows * nl; e += NT) {
    const int row = e / nl, l = e - row * nl;
    Phi[base + ((int64_t)row * nl + l) * ns + s] = F[(b.h + row) * ld + l];
  }
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
                    double dt, double dx, double nu, double* Phi, int* sq_out, int* status,
                    hipStream_t st) {
  if (nl < 3 || nl > kPhiMaxN) return hipErrorInvalidValue;
  const int mp = (nl + 15) / 16 * 16;
  const size_t lds = ((size_t)3 * mp * (mp + 1) + 8) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)ere_phi1_kernel<256>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(((size_t)3 * kPhiMaxN * (kPhiMaxN + 1) + 8) * 8));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(ere_phi1_kernel<256>, dim3((unsigned)(nb * ns)), dim3(256), lds, st, x,
                     (const EreBox*)boxes, ns, nl, rows, n, dt, dx, nu, Phi, sq_out, status);
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
  hipLaunchKernelGGL(ere_apply_kernel, ere_grid((int64_t)nb * rows * ns), dim3(256), 0, st, x, f,
                     Phi, (const EreBox*)boxes, nb, ns, nl, rows, n, y);
  return hipGetLastError();
}

}  // namespace lem
