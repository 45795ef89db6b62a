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

static inline dim3 ere_grid(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

size_t ere_box_size() { return sizeof(EreBox); }

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
