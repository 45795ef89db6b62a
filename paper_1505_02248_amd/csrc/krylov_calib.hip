// Krylov calibration kernels (gfx950).
//
// At plan time one Arnoldi run per class of blocks, on a pseudo-random probe,
// gives the Hessenberg matrix H of the largest allowed dimension; since the
// Krylov subspace of dt/nsub * A_M is the one of dt * A_M, the leading j x j
// block of H / nsub is the projection for dimension j and nsub sub-steps, and
// Saad's estimate for every (j, nsub) pair follows from exp of that block.
#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

// Calibration estimates: for block `item / (nj * ns_cand)`, Krylov dimension
// j = jlist[...] and sub-step count nsub = 2^e, the relative estimate of one
// full step: nsub * h_{j+1,j}/nsub * |e_j^T exp(H_j / nsub) e_1|.
struct EstArgs {
  const double* calib;  // per block: beta, k, H ((mc+1) x mc)
  const int* mcal;      // per block calibration dimension mc
  const int64_t* coff;  // per block offset into calib
  const int* jlist;     // candidate dimensions
  int nj;
  int n_sub_cand;       // candidates nsub = 1, 2, 4, ..., 2^(n_sub_cand-1)
  double* est;          // [block][sub][j]
};

template <int NT>
__global__ __launch_bounds__(NT) void krylov_estimate_kernel(EstArgs a) {
  extern __shared__ double smem[];
  const int item = blockIdx.x;
  const int per = a.nj * a.n_sub_cand;
  const int blk = item / per;
  const int r = item - blk * per;
  const int e = r / a.nj;
  const int j = a.jlist[r - e * a.nj];
  const int mc = a.mcal[blk];
  const double* c = a.calib + a.coff[blk];
  const int k = (int)c[1];
  double* out = a.est + item;
  if (j > mc) { if (threadIdx.x == 0) *out = INFINITY; return; }
  if (j > k) { if (threadIdx.x == 0) *out = 0.0; return; }  // invariant subspace
  const double* Hc = c + 2;
  const double inv = ldexp(1.0, -e);
  double* EA = smem;
  double* EW = EA + j * j;
  double* ER = EW + 5 * j * j;
  double* piv = ER + j * j;
  for (int idx = threadIdx.x; idx < j * j; idx += NT) {
    const int i = idx / j, q = idx - i * j;
    EA[idx] = Hc[i * mc + q] * inv;
  }
  __syncthreads();
  expm_small<NT>(EA, j, EW, ER, piv);
  if (threadIdx.x == 0) {
    // h_{j+1,j} of dt*A is scaled by 1/nsub like H; the estimate of one
    // sub-step relative to beta, times nsub sub-steps, is h_{j+1,j} |f_j|.
    const double hk = Hc[j * mc + (j - 1)];
    *out = hk * fabs(ER[(j - 1) * j]);
  }
}

// Pseudo-random probe for calibration: a counter-based hash per (block, point),
// uniform in [-1, 1).  Only used to size the Krylov dimension.
__global__ void probe_fill_kernel(double* x, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i + seed * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

hipError_t launch_krylov_estimates(const double* calib, const int* mcal,
                                   const int64_t* coff, const int* jlist, int nj,
                                   int n_sub_cand, double* est, int n_blocks,
                                   int j_max, hipStream_t st) {
  EstArgs a{calib, mcal, coff, jlist, nj, n_sub_cand, est};
  const size_t lds = (size_t)(7 * j_max * j_max + 16) * 8;
  auto fn = krylov_estimate_kernel<256>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(n_blocks * nj * n_sub_cand), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_probe_fill(double* x, int64_t n, uint64_t seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(probe_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     x, n, seed);
  return hipGetLastError();
}

}  // namespace lem
