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

// State and exponential pointers come from the block table, so the compiler
// cannot tell their address space and would emit flat accesses, which also
// count against the LDS wait counter (an LDS wait would then wait for the
// slab prefetch too).  They always point to device memory: access them as
// global.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double gload(const double* p, int64_t i) {
  return ((const gdouble*)p)[i];
}
// two adjacent doubles (16-byte aligned: i even, p 16-byte aligned)
typedef double kd2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) kd2 gkd2;
__device__ __forceinline__ kd2 gload2(const double* p, int64_t i) {
  return ((const gkd2*)p)[i >> 1];
}
__device__ __forceinline__ void gstore(double* p, int64_t i, double v) {
  ((gdouble*)p)[i] = v;
}

struct KronArgs {
  const KronBlock* blocks;
  int n_blocks;
  const double* x_in;  // used when a block carries no state pointers
  double* x_out;
  int* status;         // used when a block carries none
  int chunks;          // member groups of S per block in the grid
  int vec_ns;          // member-vector loads: the member count of every block
};

constexpr int kKronMaxL = 128;  // box side
constexpr int kKronMaxC = 64;   // core side
constexpr int kSlab = 16;       // box rows per slab (K of the second contraction)

// LDS layout (doubles), chosen so that a wave's fragment reads are 64
// consecutive doubles (or 16-double runs 128 bytes apart across a half-wave)
// and its slab stores fall on distinct banks:
//   X  slab, member s at s XM, box column lx at 16 lx, slab row r at r:
//      XM = 16 Lk + 16 (Lk = box side rounded up to 16, the K extent of the
//      first contraction; columns past the box are zero)
//   T  16 rows (slab rows) of c S values (core column, member), row stride
//      TS = 16 (mod 32)
//   Et E_x transposed, box column lx at lx ES, core row rx at rx, ES = 16
//      (mod 32) >= c rounded up to 16; zero past the core and the box.  Only
//      for member groups (S > 1): a single-state workgroup would stage E_x
//      for one member's work, so it reads its fragments from the L2 instead
//      and keeps its LDS small (more workgroups per CU)
__host__ __device__ inline int kron_lk(int L) { return (L + 15) & ~15; }
__host__ __device__ inline int kron_xm(int L) { return 16 * kron_lk(L) + 16; }
__host__ __device__ inline int kron_ts(int cs) { return (cs + 15) / 32 * 32 + 16; }
__host__ __device__ inline int kron_es(int c) { return (c + 15) / 32 * 32 + 16; }
__host__ __device__ inline size_t kron_lds_doubles(int S, int L, int c) {
  return (size_t)S * kron_xm(L) + (size_t)kSlab * kron_ts(c * S) +
         (S > 1 ? (size_t)kron_lk(L) * kron_es(c) : 0);
}

// Workgroup id g runs on XCD g % 8; the XCD-contiguous index of g numbers
// the workgroups of XCD 0 first, then those of XCD 1, ...
__device__ __forceinline__ int xcd_contiguous(int g, int count) {
  constexpr int kXcd = 8;
  const int per = count / kXcd, rem = count % kXcd;
  const int x = g % kXcd, local = g / kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// Fragment layouts (16x16x4, f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register i of lane l is D[4 i + l/16][l%16].
// (MINW: waves per SIMD the registers must allow; 4 for the ensemble shape
// at c <= 32, i.e. two eight-wave workgroups per CU, which LDS allows too.
// VEC: the member count is a multiple of S, and a thread loads all S members
// of its points with 16-byte loads instead of one member per load.)
template <int S, int NW, int MAXT, int LMAX, int MINW, bool VEC>
__global__ __launch_bounds__(NW * 64, MINW) void kron_mfma_kernel(KronArgs a) {
  constexpr int NT = NW * 64;
  static_assert(NT % (16 * S) == 0, "threads cover whole (member, slab row) sets");
  constexpr int STEP = NT / (16 * S);    // box columns between a thread's slab values
  constexpr int GMAX = LMAX / STEP;      // slab values per thread (L <= LMAX)
  extern __shared__ double smem[];
  // workgroups are dispatched to the 8 XCDs in turn; renumber them so each
  // XCD takes a contiguous run of (block, member group) pairs: the groups of
  // one block read the same cache lines of the member-fastest state, and
  // neighbouring blocks share buffer rows, in that XCD's L2
  const int g = xcd_contiguous(blockIdx.x, gridDim.x);
  const KronBlock b = a.blocks[g / a.chunks];
  if (VEC && b.ns != a.vec_ns) {  // a table built against the launch's precondition
    if (threadIdx.x == 0) atomicOr(b.status ? b.status : a.status, kStatusNonFinite);
    return;
  }
  const int s0 = (g % a.chunks) * S;
  if (s0 >= b.ns) return;
  const int sv = min(S, b.ns - s0);
  const int L = b.L, c = b.c, h = b.h, n = b.n, ns = b.ns;
  const double* x_in = b.x_in ? b.x_in : a.x_in;
  double* x_out = b.x_out ? b.x_out : a.x_out;
  const int Lk = kron_lk(L), XM = kron_xm(L);
  const int cs = c * S, TS = kron_ts(cs), ES = kron_es(c);
  const int ct = (c + 15) >> 4;          // 16-wide tiles of core rows / columns
  const int nt = (cs + 15) >> 4;         // 16-wide tiles of (core column, member)
  const int tiles = ct * nt;             // accumulator tiles of the second contraction
  double* X = smem;
  double* T = X + (size_t)S * XM;
  double* Et = T + (size_t)kSlab * TS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  // E_x core rows, transposed, into LDS; four loads in flight per thread
  constexpr bool kStageE = S > 1;
  const int etotal = kStageE ? Lk * ES : 0;
  for (int e0 = tid; e0 < etotal; e0 += 4 * NT) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + q * NT;
      const int lx = e / ES, rx = e - lx * ES;
      const bool ok = e < etotal && rx < c && lx < L;
      v[q] = gload(b.ex, ok ? (int64_t)rx * L + lx : 0);
      v[q] = ok ? v[q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (e0 + q * NT < etotal) Et[e0 + q * NT] = v[q];
  }

  // a thread's slab values: member sm, slab row rs, box columns lx0 + i STEP.
  // Loads are unconditional (from the block's own origin where a value lies
  // outside the box or the member range) and branch-free, so a thread's loads
  // of a slab are all in flight together.
  const int sm = tid % S, rs = (tid / S) & 15, lx0 = tid / (16 * S);
  const bool member_ok = sm < sv;
  const int64_t origin = ((int64_t)b.oy * n + b.ox) * ns + s0;
  auto slab_loads = [&](int ly0, double (&v)[GMAX], bool (&ok)[GMAX]) {
    const int ly = ly0 + rs;
    int gy = b.oy - h + ly;
    gy += gy < 0 ? n : 0;
    gy -= gy >= n ? n : 0;
    const int64_t row = (int64_t)gy * n;
    const bool row_ok = member_ok && ly < L;
#pragma unroll
    for (int i = 0; i < GMAX; ++i) {
      // box offsets lie within one period of the grid (h < n)
      int gx = b.ox - h + lx0 + i * STEP;
      gx += gx < 0 ? n : 0;
      gx -= gx >= n ? n : 0;
      ok[i] = row_ok && lx0 + i * STEP < L;
      v[i] = gload(x_in, ok[i] ? (row + gx) * ns + s0 + sm : origin);
    }
  };
  // VEC: thread (slab row rv, box column lv) loads the S members of columns
  // lv + i STEPV, S adjacent doubles of the member-fastest state each
  constexpr int STEPV = NT / 16;
  constexpr int GV = LMAX / STEPV;
  static_assert(!VEC || GV * S == GMAX, "member-vector loads cover the same slab");
  const int rv = tid & 15, lv = tid >> 4;
  auto slab_loads_v = [&](int ly0, double (&v)[GMAX], bool (&ok)[GMAX]) {
    const int ly = ly0 + rv;
    int gy = b.oy - h + ly;
    gy += gy < 0 ? n : 0;
    gy -= gy >= n ? n : 0;
    const int64_t row = (int64_t)gy * n;
    const bool row_ok = ly < L;
#pragma unroll
    for (int i = 0; i < GV; ++i) {
      int gx = b.ox - h + lv + i * STEPV;
      gx += gx < 0 ? n : 0;
      gx -= gx >= n ? n : 0;
      ok[i] = row_ok && lv + i * STEPV < L;
      const int64_t base = ok[i] ? (row + gx) * ns + s0 : origin;
#pragma unroll
      for (int q = 0; q < S / 2; ++q) {
        const kd2 t = gload2(x_in, base + 2 * q);
        v[i * S + 2 * q] = t.x;
        v[i * S + 2 * q + 1] = t.y;
      }
    }
  };
  double pre[GMAX];
  bool pok[GMAX];
  if constexpr (VEC) slab_loads_v(0, pre, pok);
  else slab_loads(0, pre, pok);
  kd4 acc[MAXT];
#pragma unroll
  for (int j = 0; j < MAXT; ++j) acc[j] = (kd4){0.0, 0.0, 0.0, 0.0};

  for (int ly0 = 0; ly0 < L; ly0 += kSlab) {
    // store the prefetched slab (columns up to Lk; zero outside the box)
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < GV; ++i)
        if (lv + i * STEPV < Lk) {
#pragma unroll
          for (int q = 0; q < S; ++q)
            X[q * XM + (lv + i * STEPV) * 16 + rv] = pok[i] ? pre[i * S + q] : 0.0;
        }
    } else {
#pragma unroll
      for (int i = 0; i < GMAX; ++i)
        if (lx0 + i * STEP < Lk) X[sm * XM + (lx0 + i * STEP) * 16 + rs] = pok[i] ? pre[i] : 0.0;
    }
    __syncthreads();
    // E_y fragments of this slab for the resident tiles, issued before the
    // next slab's loads (the wait for them then leaves those in flight)
    double ey[MAXT][4];
#pragma unroll
    for (int j = 0; j < MAXT; ++j) {
      const int tt = wave + NW * j;
      const int ry = (tt / nt) * 16 + lr;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int ly = ly0 + 4 * kk + lk;
        const bool ok = tt < tiles && ry < c && ly < L;
        const double v = gload(b.ey, ok ? (int64_t)ry * L + ly : 0);
        ey[j][kk] = ok ? v : 0.0;
      }
    }
    if (ly0 + kSlab < L) {
      if constexpr (VEC) slab_loads_v(ly0 + kSlab, pre, pok);
      else slab_loads(ly0 + kSlab, pre, pok);
    }
    // first contraction: one (member, 16 core columns) tile per wave at a
    // time, 16 box columns per pass
    for (int u = wave; u < S * ct; u += NW) {
      const int s = u / ct, rxt = u % ct;
      const double* xr = X + s * XM + lk * 16 + lr;
      const double* er = Et + lk * ES + rxt * 16 + lr;
      const int rx = rxt * 16 + lr;
      kd4 t = (kd4){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < Lk; k0 += 16) {
        double xa[4], eb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          xa[q] = xr[(k0 + 4 * q) * 16];
          if (kStageE) {
            eb[q] = er[(k0 + 4 * q) * ES];
          } else {
            const int lx = k0 + 4 * q + lk;
            const bool ok = rx < c && lx < L;
            const double v = gload(b.ex, ok ? (int64_t)rx * L + lx : 0);
            eb[q] = ok ? v : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) t = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[q], eb[q], t, 0, 0, 0);
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
        const int q = (tt % nt) * 16 + lr;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double bv = q < cs ? T[(4 * kk + lk) * TS + q] : 0.0;
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ey[j][kk], bv, acc[j], 0, 0, 0);
        }
      }
    }
    // no barrier here: the next slab's stores write X, which every wave has
    // finished reading (the barrier above), and T is rewritten only after
    // the next barrier, when every wave has left this loop
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
            gstore(x_out, ((int64_t)(b.oy + ry) * n + (b.ox + rx)) * ns + s0 + s, y);
          }
        }
      }
    }
  }
  if (bad) atomicOr(b.status ? b.status : a.status, kStatusNonFinite);
}

int kron_max_side() { return kKronMaxL; }
int kron_max_core() { return kKronMaxC; }

template <int S, int NW, int MAXT, int LMAX, int MINW, bool VEC>
static hipError_t launch_kron_shape(const KronBlock* blocks, int n_blocks, int max_ns, int max_L,
                                    int max_c, const double* x_in, double* x_out, int* status,
                                    hipStream_t st) {
  const int chunks = (max_ns + S - 1) / S;
  const size_t lds = kron_lds_doubles(S, max_L, max_c) * sizeof(double);
  auto fn = kron_mfma_kernel<S, NW, MAXT, LMAX, MINW, VEC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)((int64_t)n_blocks * chunks)), dim3(NW * 64), lds, st,
                     KronArgs{blocks, n_blocks, x_in, x_out, status, chunks, VEC ? max_ns : 0});
  return hipGetLastError();
}

// Blocks of one launch may differ in core side (<= max_c <= 64) and box side
// (<= max_L <= 128); with more than one member they share the member count
// max_ns (single-state launches may mix any).  Shapes (members per workgroup
// S, waves, resident tiles per wave = ceil((c/16)^2 S / waves), box side
// bound of the prefetch registers):
//   ensembles, c <= 32, L <= 64:  S = 4, 8 waves, 2 tiles
//   other ensembles:              S = 2, 8 waves, 4 tiles
//   single states:                S = 1, 4 waves, 1 tile (c <= 32) or 4
// Member counts that S divides use 16-byte member-vector loads.
hipError_t launch_kron(const KronBlock* blocks, int n_blocks, int max_ns, int max_L, int max_c,
                       const double* x_in, double* x_out, int* status, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (max_L > kKronMaxL || max_L < 1 || max_ns < 1 || max_c < 1 || max_c > kKronMaxC)
    return hipErrorInvalidValue;
  if (max_ns >= 4 && max_c <= 32 && max_L <= 64) {
    if (max_ns % 4 == 0)
      return launch_kron_shape<4, 8, 2, 64, 4, true>(blocks, n_blocks, max_ns, max_L, max_c,
                                                     x_in, x_out, status, st);
    return launch_kron_shape<4, 8, 2, 64, 4, false>(blocks, n_blocks, max_ns, max_L, max_c, x_in,
                                                    x_out, status, st);
  }
  if (max_ns >= 2) {
    if (max_ns % 2 == 0)
      return launch_kron_shape<2, 8, 4, kKronMaxL, 1, true>(blocks, n_blocks, max_ns, max_L,
                                                            max_c, x_in, x_out, status, st);
    return launch_kron_shape<2, 8, 4, kKronMaxL, 1, false>(blocks, n_blocks, max_ns, max_L, max_c,
                                                           x_in, x_out, status, st);
  }
  if (max_c <= 32)
    return launch_kron_shape<1, 4, 1, kKronMaxL, 1, false>(blocks, n_blocks, max_ns, max_L, max_c,
                                                           x_in, x_out, status, st);
  return launch_kron_shape<1, 4, 4, kKronMaxL, 1, false>(blocks, n_blocks, max_ns, max_L, max_c,
                                                         x_in, x_out, status, st);
}

}  // namespace lem
