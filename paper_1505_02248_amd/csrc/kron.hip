// Stored local exponentials in Kronecker-factored form (gfx950).
//
// On a rectangular box of a 2D constant-coefficient operator the local
// matrix of the local problem (4) (section 3: couplings leaving the box
// dropped) is the Kronecker sum A_M = I (x) A_x + A_y (x) I of two tridiagonal
// 1D matrices, which commute, so exp(dt A_M) = exp(dt A_y) (x) exp(dt A_x)
// exactly.  The core rows of the local result are then
//     Y = E_y[core rows, :] * X * E_x[core rows, :]^T
// for the box values X (L x L, y rows, x columns): two small contractions
// instead of one with the (c^2 x L^2) core block, and the stored data are two
// c x L matrices.  One workgroup per (member, block): the gathered box in LDS,
// then, per group of 16 core columns, T = X E_x^T (L x 16) in LDS and
// Y = E_y T written to the core (step 3).
#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

struct KronArgs {
  const KronBlock* blocks;
  int n_blocks;
  const double* x_in;  // used when a block carries no state pointers
  double* x_out;
  int* status;         // used when a block carries none
  int max_ns;          // members per block in the grid (blocks with fewer skip the rest)
};

constexpr int kKronCols = 16;   // core columns per pass
constexpr int kKronMaxL = 128;  // box side (LDS: L (L + 1) + L (16 + 1) doubles)

__host__ __device__ inline size_t kron_lds_doubles(int L) {
  return (size_t)L * (L + 1) + (size_t)L * (kKronCols + 1);
}

template <int NT>
__global__ __launch_bounds__(NT) void kron_apply_kernel(KronArgs a) {
  extern __shared__ double smem[];
  // consecutive workgroups take consecutive members of one block: they read
  // the same cache lines of the member-fastest state
  const KronBlock b = a.blocks[blockIdx.x / a.max_ns];
  const int s = blockIdx.x % a.max_ns;
  if (s >= b.ns) return;
  const int L = b.L, c = b.c, h = b.h, n = b.n, ns = b.ns;
  const double* x_in = b.x_in ? b.x_in : a.x_in;
  double* x_out = b.x_out ? b.x_out : a.x_out;
  const int XS = L + 1;  // padded LDS row
  double* X = smem;
  double* T = smem + (size_t)L * XS;
  const int tid = threadIdx.x;
  // gather the box (periodic wrap of the global grid)
  for (int e = tid; e < L * L; e += NT) {
    const int ly = e / L, lx = e - ly * L;
    const int gx = wrap(b.ox - h + lx, n), gy = wrap(b.oy - h + ly, n);
    X[ly * XS + lx] = x_in[((int64_t)gy * n + gx) * ns + s];
  }
  __syncthreads();
  bool bad = false;
  for (int rx0 = 0; rx0 < c; rx0 += kKronCols) {
    const int w = min(kKronCols, c - rx0);
    // T[ly][j] = sum_lx X[ly][lx] E_x[rx0 + j][lx]
    for (int e = tid; e < L * w; e += NT) {
      const int ly = e / w, j = e - ly * w;
      const double* ex = b.ex + (int64_t)(rx0 + j) * L;
      const double* xr = X + ly * XS;
      double t0 = 0.0, t1 = 0.0;
      int lx = 0;
      for (; lx + 1 < L; lx += 2) {
        t0 = fma(xr[lx], ex[lx], t0);
        t1 = fma(xr[lx + 1], ex[lx + 1], t1);
      }
      if (lx < L) t0 = fma(xr[lx], ex[lx], t0);
      T[ly * (kKronCols + 1) + j] = t0 + t1;
    }
    __syncthreads();
    // Y[ry][rx0 + j] = sum_ly E_y[ry][ly] T[ly][j]
    for (int e = tid; e < c * w; e += NT) {
      const int ry = e / w, j = e - ry * w;
      const double* ey = b.ey + (int64_t)ry * L;
      double t0 = 0.0, t1 = 0.0;
      int ly = 0;
      for (; ly + 1 < L; ly += 2) {
        t0 = fma(ey[ly], T[ly * (kKronCols + 1) + j], t0);
        t1 = fma(ey[ly + 1], T[(ly + 1) * (kKronCols + 1) + j], t1);
      }
      if (ly < L) t0 = fma(ey[ly], T[ly * (kKronCols + 1) + j], t0);
      const double y = t0 + t1;
      bad |= !isfinite(y);
      x_out[((int64_t)(b.oy + ry) * n + (b.ox + rx0 + j)) * ns + s] = y;
    }
    __syncthreads();
  }
  if (bad) atomicOr(b.status ? b.status : a.status, kStatusNonFinite);
}

size_t kron_lds_bytes(int L) { return kron_lds_doubles(L) * sizeof(double); }
int kron_max_side() { return kKronMaxL; }

hipError_t launch_kron(const KronBlock* blocks, int n_blocks, int max_ns, int max_L,
                       const double* x_in, double* x_out, int* status, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (max_L > kKronMaxL || max_L < 1 || max_ns < 1) return hipErrorInvalidValue;
  const size_t lds = kron_lds_bytes(max_L);
  auto fn = kron_apply_kernel<256>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)((int64_t)n_blocks * max_ns)), dim3(256), lds, st,
                     KronArgs{blocks, n_blocks, x_in, x_out, status, max_ns});
  return hipGetLastError();
}

}  // namespace lem
