// Batched Arnoldi-Krylov LEM step (gfx950).
//
// One workgroup advances one region M_i (one ensemble member) of the
// overlapping decomposition of section 3 by one time step:
//   1. gather the local state v = u^n restricted to the box (core + buffer);
//   2. for each of nsub equal sub-steps, build the Krylov basis V_m of
//      K_m(dt_sub A_M, v) by Arnoldi (classical Gram-Schmidt with one full
//      re-orthogonalization pass), the stencil product of the local problem (4)
//      applied on the box with couplings to outside nodes dropped; then
//      v <- beta V_m exp(H_m) e_1 (the Krylov action of section 4.3), with
//      exp(H_m) by Pade scaling and squaring in LDS;
//   3. write the core rows of v into u^{n+1} (step 3 of section 3).
// Saad's estimate beta * h_{m+1,m} * |e_m^T exp(H_m) e_1| is computed for
// every sub-step and latched into the status word when above tolerance.
//
// The basis lives in LDS when (m+1) * |M_i| doubles fit next to the Hessenberg
// work space, and otherwise in a per-block slice of device memory that the
// workgroup streams (L2/HBM).
#include "lem_device.hpp"

namespace lem {


// LDS layout (doubles), shared with the host sizing routine.
__host__ __device__ inline int64_t krylov_lds_doubles(int NT, int m, int nloc,
                                                      bool vlds) {
  int64_t d = 0;
  d += (int64_t)(m + 1) * m;      // H
  d += 2 * (m + 1);               // dot results (two passes)
  d += (NT / 64) * 8 + 8;         // reduction scratch
  d += NT / 64 + 8;               // pivot / misc
  d += 7 * (int64_t)m * m;        // expm: A, W(5), R
  if (vlds) d += (int64_t)(m + 1) * nloc;
  return d;
}

template <int NT, int PMAX, bool VLDS>
__global__ __launch_bounds__(NT) void krylov_lem_kernel(KrylovArgs a) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int s = blockIdx.y;
  const KBlock b = a.blocks[blockIdx.x];
  const int m = b.m;
  const int nloc = b.Lx * b.Ly;

  double* H = smem;                       // (m+1) x m, H[i*m + j]
  double* hv = H + (m + 1) * m;           // pass-1 dots
  double* hv2 = hv + (m + 1);             // pass-2 dots
  double* red = hv2 + (m + 1);            // (NT/64)*8 + 8
  double* piv = red + (NT / 64) * 8 + 8;  // NT/64 + 8
  double* EA = piv + NT / 64 + 8;         // m*m
  double* EW = EA + m * m;                // 5*m*m
  double* ER = EW + 5 * m * m;            // m*m
  const double* x_in = b.xin ? b.xin : a.x_in;
  double* x_out = b.xout ? b.xout : a.x_out;
  double* V;
  if (VLDS) {
    V = ER + m * m;
  } else {
    V = (b.vwork ? b.vwork : a.vwork + b.v_off) + (int64_t)s * (m + 1) * nloc;
  }

  // Points owned by this thread and their box coordinates.
  int lxs[PMAX], lys[PMAX];
  bool live[PMAX];
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    const int l = tid + p * NT;
    live[p] = l < nloc;
    lys[p] = live[p] ? l / b.Lx : 0;
    lxs[p] = live[p] ? l - lys[p] * b.Lx : 0;
  }
  const bool varcoef = b.mu_off >= 0;
  const double* mux = (b.coef ? b.coef : a.coef) + (varcoef ? b.mu_off : 0);
  const int64_t Ng = (b.ndim == 1) ? b.n : (int64_t)b.n * b.n;
  const double* muy = mux + Ng;

  // 1. gather
  double cur[PMAX];
#pragma unroll
  for (int p = 0; p < PMAX; ++p)
    cur[p] = live[p] ? x_in[b.x_off + gather_index(b, lxs[p], lys[p]) * b.ns + s] : 0.0;

  double nrm0 = 0.0;
#pragma unroll
  for (int p = 0; p < PMAX; ++p) nrm0 = fma(cur[p], cur[p], nrm0);
  const double beta0 = sqrt(wg_sum1<NT>(nrm0, red));
  double worst = 0.0;
  bool bad = !isfinite(beta0);

  const int nsub = (a.mode == 1) ? 1 : b.nsub;
  for (int sub = 0; sub < nsub; ++sub) {
    double beta = beta0;
    if (sub > 0) {
      double t = 0.0;
#pragma unroll
      for (int p = 0; p < PMAX; ++p) t = fma(cur[p], cur[p], t);
      beta = sqrt(wg_sum1<NT>(t, red));
    }
    if (!(beta > 0.0) || !isfinite(beta)) {
      if (!isfinite(beta)) bad = true;
      break;  // zero (or broken) local state stays as it is
    }
    const double ib = 1.0 / beta;
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
      if (live[p]) V[tid + p * NT] = cur[p] * ib;
    for (int idx = tid; idx < (m + 1) * m; idx += NT) H[idx] = 0.0;
    __syncthreads();

    int k = m;
    for (int j = 0; j < m; ++j) {
      const double* vj = V + (int64_t)j * nloc;
      double w[PMAX];
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        double r = 0.0;
        if (live[p]) {
          const int l = tid + p * NT, lx = lxs[p], ly = lys[p];
          double c0, cW, cE, cS, cN;
          if (!varcoef) {
            c0 = b.w0; cW = b.wW; cE = b.wE; cS = b.wS; cN = b.wN;
          } else {
            const int gx = wrap(b.ox - b.h + lx, b.n);
            const int gy = (b.ndim == 1) ? 0 : wrap(b.oy - b.h + ly, b.n);
            const int64_t g = (int64_t)gy * b.n + gx;
            const double me = mux[g];
            const double mw = mux[(int64_t)gy * b.n + wrap(gx - 1, b.n)];
            double mn = 0.0, ms = 0.0;
            if (b.ndim == 2) {
              mn = muy[g];
              ms = muy[(int64_t)wrap(gy - 1, b.n) * b.n + gx];
            }
            const double sc = b.sub_scale;
            c0 = -(me + mw + mn + ms) * sc;
            cW = fma(mw, sc, b.chx);
            cE = fma(me, sc, -b.chx);
            cS = fma(ms, sc, b.chy);
            cN = fma(mn, sc, -b.chy);
          }
          r = c0 * vj[l];
          if (lx > 0) r = fma(cW, vj[l - 1], r);
          if (lx < b.Lx - 1) r = fma(cE, vj[l + 1], r);
          if (ly > 0) r = fma(cS, vj[l - b.Lx], r);
          if (ly < b.Ly - 1) r = fma(cN, vj[l + b.Lx], r);
        }
        w[p] = r;
      }
      // Two classical Gram-Schmidt passes.
      for (int pass = 0; pass < 2; ++pass) {
        double* dots = pass == 0 ? hv : hv2;
        for (int i0 = 0; i0 <= j; i0 += 8) {
          const int cnt = min(8, j + 1 - i0);
          double part[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            double t = 0.0;
            if (q < cnt) {
              const double* vi = V + (int64_t)(i0 + q) * nloc;
#pragma unroll
              for (int p = 0; p < PMAX; ++p)
                if (live[p]) t = fma(vi[tid + p * NT], w[p], t);
            }
            part[q] = t;
          }
          wg_sum<NT, 8>(part, cnt, red, dots + i0);
        }
        for (int i = 0; i <= j; ++i) {
          const double hi = dots[i];
          const double* vi = V + (int64_t)i * nloc;
#pragma unroll
          for (int p = 0; p < PMAX; ++p)
            if (live[p]) w[p] = fma(-hi, vi[tid + p * NT], w[p]);
        }
      }
      double t = 0.0;
#pragma unroll
      for (int p = 0; p < PMAX; ++p) t = fma(w[p], w[p], t);
      const double hn = sqrt(wg_sum1<NT>(t, red));
      double hs = 0.0;
      for (int i = 0; i <= j; ++i) {
        const double hij = hv[i] + hv2[i];
        hs = fma(hij, hij, hs);
        if (tid == 0) H[i * m + j] = hij;
      }
      if (tid == 0) H[(j + 1) * m + j] = hn;
      if (!(hn > 1e-14 * sqrt(hs + hn * hn))) {  // happy breakdown (or zero)
        k = j + 1;
        __syncthreads();
        break;
      }
      const double ih = 1.0 / hn;
      double* vn = V + (int64_t)(j + 1) * nloc;
#pragma unroll
      for (int p = 0; p < PMAX; ++p)
        if (live[p]) vn[tid + p * NT] = w[p] * ih;
      __syncthreads();
    }

    if (a.mode == 1) {
      // Calibration: export beta, k and H.
      double* out = a.calib + ((int64_t)b.diag * b.ns + s) * (2 + (m + 1) * m);
      for (int idx = tid; idx < (m + 1) * m; idx += NT) out[2 + idx] = H[idx];
      if (tid == 0) { out[0] = beta; out[1] = (double)k; }
      return;
    }

    // exp(H_k) e_1
    for (int idx = tid; idx < k * k; idx += NT) {
      const int i = idx / k, jj = idx - i * k;
      EA[idx] = H[i * m + jj];
    }
    __syncthreads();
    expm_small<NT>(EA, k, EW, ER, piv);
    const double hk = H[k * m + (k - 1)];
    const double est = beta * hk * fabs(ER[(k - 1) * k]) / beta0;
    worst += est;  // the step's estimate is the sum over its sub-steps
    // v <- beta V_k f
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      if (!live[p]) continue;
      double acc = 0.0;
      for (int i = 0; i < k; ++i)
        acc = fma(ER[i * k], V[(int64_t)i * nloc + tid + p * NT], acc);
      cur[p] = beta * acc;
    }
    __syncthreads();
  }

  // 3. core overwrite
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    if (!live[p]) continue;
    const int lx = lxs[p], ly = lys[p];
    const int rx = lx - b.h;
    const int ry = (b.ndim == 1) ? ly : ly - b.h;
    if (rx < 0 || rx >= b.cx || ry < 0 || ry >= b.cy) continue;
    const int64_t g = (b.ndim == 1) ? (int64_t)(b.ox + rx)
                                    : (int64_t)(b.oy + ry) * b.n + (b.ox + rx);
    if (!isfinite(cur[p])) bad = true;
    x_out[b.x_off + g * b.ns + s] = cur[p];
  }
  if (bad) atomicOr(a.status, kStatusNonFinite);
  if (tid == 0) {
    a.diag[(int64_t)b.diag * b.ns + s] = worst;
    if (!(worst <= b.tol)) atomicOr(a.status, kStatusNotConverged);
  }
}

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

}  // namespace lem

// ------------------------------------------------------------------ launch --
#include "lem_launch.h"

namespace lem {

template <int NT, int PMAX, bool VLDS>
static hipError_t launch_k(const KrylovArgs& a, int ns, size_t lds, hipStream_t st) {
  auto fn = krylov_lem_kernel<NT, PMAX, VLDS>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(a.n_blocks, ns), dim3(NT), lds, st, a);
  return hipGetLastError();
}

// Launch shape for a local box of nloc points: workgroup size and the
// per-thread point count (template instantiation) that covers it.
void krylov_config(int ndim, int nloc, int* nt, int* pmax) {
  if (ndim == 1 && nloc <= 128) { *nt = 64; *pmax = 2; return; }
  if (ndim == 1 && nloc <= 512) { *nt = 64; *pmax = 8; return; }
  if (nloc <= 1024) { *nt = 256; *pmax = 4; return; }
  if (nloc <= 4096) { *nt = 256; *pmax = 16; return; }
  if (nloc <= 10240) { *nt = 512; *pmax = 20; return; }
  *nt = 0; *pmax = 0;
}

size_t krylov_lds_bytes(int nt, int m, int nloc, bool vlds) {
  return (size_t)krylov_lds_doubles(nt, m, nloc, vlds) * 8;
}

hipError_t launch_krylov(const KBlock* blocks, int n_blocks, int ns, int nt, int pmax,
                         bool vlds, size_t lds, const double* x_in, double* x_out,
                         const double* coef, double* vwork, double* diag, int* status,
                         double* calib, int mode, hipStream_t st) {
  KrylovArgs a{blocks, x_in, x_out, coef, vwork, diag, status, calib, mode, n_blocks};
  if (n_blocks == 0) return hipSuccess;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (nt == 64 && pmax == 2)
    return vlds ? launch_k<64, 2, true>(a, ns, lds, st) : launch_k<64, 2, false>(a, ns, lds, st);
  if (nt == 64 && pmax == 8)
    return vlds ? launch_k<64, 8, true>(a, ns, lds, st) : launch_k<64, 8, false>(a, ns, lds, st);
  if (nt == 256 && pmax == 4)
    return vlds ? launch_k<256, 4, true>(a, ns, lds, st) : launch_k<256, 4, false>(a, ns, lds, st);
  if (nt == 256 && pmax == 16)
    return vlds ? launch_k<256, 16, true>(a, ns, lds, st) : launch_k<256, 16, false>(a, ns, lds, st);
  if (nt == 512 && pmax == 20 && !vlds) return launch_k<512, 20, false>(a, ns, lds, st);
  return hipErrorInvalidValue;
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
