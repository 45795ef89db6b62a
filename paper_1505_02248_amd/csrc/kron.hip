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
// c x L matrices.
//
// Both contractions run on FP64 MFMA (v_mfma_f64_16x16x4).  A workgroup
// takes one block and S members of it and walks the box in slabs of 16 rows:
//   gather   X[s][r][lx]   = x(row ly0 + r, column lx, member s)   (LDS)
//   first    T[r][rx, s]   = sum_lx X[s][r][lx] E_x[rx][lx]        (LDS)
//   second   Y[ry][rx, s] += sum_r  E_y[ry][ly0 + r] T[r][rx, s]   (registers)
// and writes the core of Y at the end (step 3).  LDS holds one slab, so the
// box side only bounds the loop, and S members of one point are S adjacent
// doubles of the member-fastest state, read together.
#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

typedef double kd4 __attribute__((ext_vector_type(4)));

struct KronArgs {
  const KronBlock* blocks;
  int n_blocks;
  const double* x_in;  // used when a block carries no state pointers
  double* x_out;
  int* status;         // used when a block carries none
  int chunks;          // member groups of S per block in the grid
};

constexpr int kKronMaxL = 128;  // box side
constexpr int kKronMaxC = 64;   // core side
constexpr int kSlab = 16;       // box rows per slab (K of the second contraction)

// LDS doubles for S members: the slab S x 16 x (L rounded to 4, plus one)
// and T 16 x (c S + 1)
__host__ __device__ inline int kron_xs(int L) { return ((L + 3) & ~3) + 1; }
__host__ __device__ inline size_t kron_lds_doubles(int S, int L, int c) {
  return (size_t)S * kSlab * kron_xs(L) + (size_t)kSlab * (c * S + 1);
}

// Fragment layouts (16x16x4, f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register i of lane l is D[4 i + l/16][l%16].
template <int S, int NW, int MAXT>
__global__ __launch_bounds__(NW * 64) void kron_mfma_kernel(KronArgs a) {
  extern __shared__ double smem[];
  const KronBlock b = a.blocks[blockIdx.x / a.chunks];
  const int s0 = (blockIdx.x % a.chunks) * S;
  if (s0 >= b.ns) return;
  const int sv = min(S, b.ns - s0);
  const int L = b.L, c = b.c, h = b.h, n = b.n, ns = b.ns;
  const double* x_in = b.x_in ? b.x_in : a.x_in;
  double* x_out = b.x_out ? b.x_out : a.x_out;
  const int Lp = (L + 3) & ~3, XS = Lp + 1;
  const int cs = c * S, TS = cs + 1;
  double* X = smem;
  double* T = smem + (size_t)S * kSlab * XS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int ct = (c + 15) >> 4;          // 16-wide tiles of core rows / columns
  const int nt = (cs + 15) >> 4;         // 16-wide tiles of (core column, member)
  const int tiles = ct * nt;             // accumulator tiles of the second contraction
  kd4 acc[MAXT];
#pragma unroll
  for (int j = 0; j < MAXT; ++j) acc[j] = (kd4){0.0, 0.0, 0.0, 0.0};

  for (int ly0 = 0; ly0 < L; ly0 += kSlab) {
    // gather the slab, members fastest (S adjacent doubles per point)
    for (int e = tid; e < kSlab * Lp * S; e += NW * 64) {
      const int s = e % S, rest = e / S;
      const int lx = rest % Lp, r = rest / Lp;
      const int ly = ly0 + r;
      double v = 0.0;
      if (ly < L && lx < L && s < sv) {
        const int gx = wrap(b.ox - h + lx, n), gy = wrap(b.oy - h + ly, n);
        v = x_in[((int64_t)gy * n + gx) * ns + s0 + s];
      }
      X[(s * kSlab + r) * XS + lx] = v;
    }
    __syncthreads();
    // first contraction: one (member, 16 core columns) tile per wave at a time
    for (int u = wave; u < S * ct; u += NW) {
      const int s = u / ct, rx = (u % ct) * 16 + lr;
      const double* xr = X + (s * kSlab + lr) * XS + lk;
      const double* exr = b.ex + (int64_t)rx * L + lk;
      kd4 t = (kd4){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < Lp; k0 += 4) {
        const double bv = (rx < c && k0 + lk < L) ? exr[k0] : 0.0;
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[k0], bv, t, 0, 0, 0);
      }
      if (rx < c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) T[(4 * i + lk) * TS + rx * S + s] = t[i];
      }
    }
    __syncthreads();
    // second contraction over the slab's 16 rows into the resident tiles
#pragma unroll
    for (int j = 0; j < MAXT; ++j) {
      const int tt = wave + NW * j;
      if (tt < tiles) {
        const int ry = (tt / nt) * 16 + lr, q = (tt % nt) * 16 + lr;
        const double* eyr = b.ey + (int64_t)ry * L + ly0 + lk;
#pragma unroll
        for (int kk = 0; kk < kSlab; kk += 4) {
          const double av = (ry < c && ly0 + kk + lk < L) ? eyr[kk] : 0.0;
          const double bv = q < cs ? T[(kk + lk) * TS + q] : 0.0;
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
        }
      }
    }
    // the next gather writes X only; T is rewritten after the barrier that
    // follows it, when every wave has left this loop
  }
  // core write (step 3)
  bool bad = false;
#pragma unroll
  for (int j = 0; j < MAXT; ++j) {
    const int tt = wave + NW * j;
    if (tt < tiles) {
      const int q = (tt % nt) * 16 + lr;
      const int rx = q / S, s = q % S;
      if (q < cs && s < sv) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ry = (tt / nt) * 16 + 4 * i + lk;
          if (ry < c) {
            const double y = acc[j][i];
            bad |= !isfinite(y);
            x_out[((int64_t)(b.oy + ry) * n + (b.ox + rx)) * ns + s0 + s] = y;
          }
        }
      }
    }
  }
  if (bad) atomicOr(b.status ? b.status : a.status, kStatusNonFinite);
}

int kron_max_side() { return kKronMaxL; }
int kron_max_core() { return kKronMaxC; }

template <int S, int NW, int MAXT>
static hipError_t launch_kron_shape(const KronBlock* blocks, int n_blocks, int max_ns, int max_L,
                                    int max_c, const double* x_in, double* x_out, int* status,
                                    hipStream_t st) {
  const int chunks = (max_ns + S - 1) / S;
  const size_t lds = kron_lds_doubles(S, max_L, max_c) * sizeof(double);
  auto fn = kron_mfma_kernel<S, NW, MAXT>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)((int64_t)n_blocks * chunks)), dim3(NW * 64), lds, st,
                     KronArgs{blocks, n_blocks, x_in, x_out, status, chunks});
  return hipGetLastError();
}

// Blocks of one launch may differ in core side (<= max_c <= 64), box side
// (<= max_L <= 128) and member count (<= max_ns).  Ensembles take four members
// per workgroup (eight waves hold the 4 x 4 x 16 tiles of a 64-point core),
// single states one (four waves).
hipError_t launch_kron(const KronBlock* blocks, int n_blocks, int max_ns, int max_L, int max_c,
                       const double* x_in, double* x_out, int* status, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (max_L > kKronMaxL || max_L < 1 || max_ns < 1 || max_c < 1 || max_c > kKronMaxC)
    return hipErrorInvalidValue;
  // resident tiles per wave: ceil((c/16)^2 S / waves); cores up to 32 need a
  // quarter of those of 64 (fewer registers, two workgroups per CU)
  if (max_ns >= 4) {
    if (max_c <= 32)
      return launch_kron_shape<4, 8, 2>(blocks, n_blocks, max_ns, max_L, max_c, x_in, x_out,
                                        status, st);
    return launch_kron_shape<4, 8, 8>(blocks, n_blocks, max_ns, max_L, max_c, x_in, x_out,
                                      status, st);
  }
  if (max_c <= 32)
    return launch_kron_shape<1, 4, 1>(blocks, n_blocks, max_ns, max_L, max_c, x_in, x_out,
                                      status, st);
  return launch_kron_shape<1, 4, 4>(blocks, n_blocks, max_ns, max_L, max_c, x_in, x_out, status,
                                    st);
}

}  // namespace lem
