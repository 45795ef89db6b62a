// Global Krylov action exp(dt A) u on the whole periodic grid (gfx950); with
// a forcing g constant over the step, the action of the augmented matrix
// [[dt A, dt g], [0, 0]] on [u; 1] (one extra coordinate per state).
//
// This is the "standard exponential method" with a single domain (D = 1) that
// the paper compares LEM against, computed by the Krylov method of Saad
// (section 4.3) for every member of an ensemble at once.  State and basis are
// stored DOF-major with the ensemble index fastest (x[pt * ns + s]), so every
// kernel streams contiguous memory.  Each Arnoldi column takes three passes
// over the grid -- stencil product fused with normalization and the first
// Gram-Schmidt dots, update fused with the re-orthogonalization dots, update
// fused with the norm -- each followed by a deterministic two-stage reduction
// (per-workgroup partials, then one workgroup per (row, state)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

struct GlobalOp {
  double w0, wW, wE, wS, wN;  // constant weights of dt_sub*A (mu == null)
  double chx, chy, sub_scale; // variable-nu form
  const double* mux;          // face-mu arrays (dt-scaled), or null
  const double* muy;
  const double* ax;           // face velocity coefficients (dt a / (2 dx)), or null
  const double* ay;
  int n, ndim;
  // forced step: point Npts is the augmented coordinate of [[dt A, dt g],
  // [0, 0]] (zero row); its column is gscale * g
  int aug;
  int64_t Npts;
  double gscale;
  const double* force;
};

__device__ __forceinline__ double gstencil(const GlobalOp& o, const double* X, int64_t pt,
                                           int ns, int s) {
  if (o.aug && pt == o.Npts) return 0.0;
  const int n = o.n;
  int64_t gx, gy;
  if (o.ndim == 1) { gx = pt; gy = 0; } else { gy = pt / n; gx = pt - gy * n; }
  const int64_t xm = (gx == 0) ? n - 1 : gx - 1, xp = (gx == n - 1) ? 0 : gx + 1;
  double c0 = o.w0, cW = o.wW, cE = o.wE, cS = o.wS, cN = o.wN;
  if (o.mux) {
    const double me = o.mux[gy * n + gx], mw = o.mux[gy * n + xm];
    double mn = 0.0, ms = 0.0;
    if (o.ndim == 2) {
      const int64_t ym = (gy == 0) ? n - 1 : gy - 1;
      mn = o.muy[gy * n + gx];
      ms = o.muy[ym * n + gx];
    }
    const double sc = o.sub_scale;
    c0 = -(me + mw + mn + ms) * sc;
    if (o.ax) {  // conservative centered advection by face velocities
      const double ae = o.ax[gy * n + gx] * sc, aw = o.ax[gy * n + xm] * sc;
      double an = 0.0, as = 0.0;
      if (o.ndim == 2) {
        const int64_t ym = (gy == 0) ? n - 1 : gy - 1;
        an = o.ay[gy * n + gx] * sc;
        as = o.ay[ym * n + gx] * sc;
      }
      c0 -= (ae - aw) + (an - as);
      cW = fma(mw, sc, aw);
      cE = fma(me, sc, -ae);
      cS = fma(ms, sc, as);
      cN = fma(mn, sc, -an);
    } else {
      cW = fma(mw, sc, o.chx);
      cE = fma(me, sc, -o.chx);
      cS = fma(ms, sc, o.chy);
      cN = fma(mn, sc, -o.chy);
    }
  }
  double r = c0 * X[pt * ns + s];
  r = fma(cW, X[(gy * n + xm) * ns + s], r);
  r = fma(cE, X[(gy * n + xp) * ns + s], r);
  if (o.ndim == 2) {
    const int64_t ym = (gy == 0) ? n - 1 : gy - 1, yp = (gy == n - 1) ? 0 : gy + 1;
    r = fma(cS, X[(ym * n + gx) * ns + s], r);
    r = fma(cN, X[(yp * n + gx) * ns + s], r);
  }
  if (o.aug) r = fma(o.gscale * o.force[pt * ns + s], X[o.Npts * ns + s], r);
  return r;
}

// Augmented state [x; 1] (forced steps) and back.
__global__ void g_aug_in(const double* x, double* xa, int64_t nx, int ns) {
  const int64_t total = nx + ns;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    xa[e] = e < nx ? x[e] : 1.0;
}

__global__ void g_copy(const double* a, double* b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

struct GArgs {
  GlobalOp op;
  double* V;        // (m+1) vectors of N*ns
  double* W;        // unnormalized next vector
  double* Wt;       // current w
  double* part;     // [G][K][ns] partial sums
  const double* inv;   // per state scale of W (1/beta or 1/h_{j,j-1})
  const double* hco;   // [K][ns] coefficients for an update pass
  int64_t N;        // grid points
  int ns, j;
};

// Reduces cnt <= K per-thread values (indexed by the thread's state) into
// part[blockIdx.x][q][s] (row stride K).  ns must divide 256, so that threads
// of one workgroup cover 256/ns points of every state; lanes l and l ^ off of
// a wave hold the same state whenever ns <= off.  Chunks of 8 values keep the
// LDS footprint at 16 KB.
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], int cnt, int ns,
                                               double* part, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if constexpr (K <= 32) {
    if (ns == 1) {
      // one state: reduce-scatter the K values over the wave (lane l ends
      // with the wave total of value l / (64 / K)), then add the 4 waves
      const double r = wave_reduce_scatter<K>(v);
      constexpr int LPV = 64 / K;
      if (lane % LPV == 0) red[wv * K + lane / LPV] = r;
      __syncthreads();
      for (int q = tid; q < cnt; q += 256)
        part[(int64_t)blockIdx.x * K + q] = red[q] + red[K + q] + red[2 * K + q] + red[3 * K + q];
      __syncthreads();
      return;
    }
  }
  for (int off = 32; off >= ns && off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < K; ++q)
      if (q < cnt) v[q] += __shfl_xor(v[q], off, 64);
  }
  const int lanes = ns < 64 ? ns : 64;  // distinct states per wave
  for (int q0 = 0; q0 < cnt; q0 += 8) {
    const int c = min(8, cnt - q0);
    if (lane < lanes) {
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (q >= q0 && q < q0 + c) red[(wv * 8 + (q - q0)) * 64 + lane] = v[q];
    }
    __syncthreads();
    for (int idx = tid; idx < c * ns; idx += 256) {
      const int q = idx / ns, s = idx - q * ns;
      double t = 0.0;
      for (int w = 0; w < 4; ++w) {
        if (ns >= 64) {
          if ((w * 64) % ns == s - (s % 64)) t += red[(w * 8 + q) * 64 + (s % 64)];
        } else {
          t += red[(w * 8 + q) * 64 + s];
        }
      }
      part[((int64_t)blockIdx.x * K + q0 + q) * ns + s] = t;
    }
    __syncthreads();
  }
}

__global__ void g_zero_kernel(double* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// Clears the Hessenberg matrices (entries below the subdiagonal are never
// written by the column updates).
static void zero_h(const GlobalWork& w, hipStream_t st) {
  const int64_t n = (int64_t)w.ns * (w.m + 1) * w.m;
  hipLaunchKernelGGL(g_zero_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)),
                     dim3(256), 0, st, w.H, n);
}

// beta, k = m and H per state, for the calibration of (m, sub-steps).
__global__ void g_export_kernel(const double* H, const double* beta, int m, double* calib) {
  const int s = blockIdx.x;
  double* out = calib + (int64_t)s * (2 + (m + 1) * m);
  const double* Hs = H + (int64_t)s * (m + 1) * m;
  for (int i = threadIdx.x; i < (m + 1) * m; i += blockDim.x) out[2 + i] = Hs[i];
  if (threadIdx.x == 0) { out[0] = beta[s]; out[1] = (double)m; }
}

// The passes take K >= j + 1 basis vectors (the launcher picks the smallest
// of 4, 8, 16, 32, 49).  Every basis load is unconditional, its vector index
// clamped to a valid one, and rows past the current ones are masked out of
// the arithmetic afterwards: all K loads of a point are in flight before the
// first use instead of one guarded load at a time.

// Pass 1: v_j = W * inv (stored into V_j), w = dt A v_j (into Wt), partial
// dots <v_i, w> for i <= j.
template <int K>
__global__ __launch_bounds__(256) void g_spmv_dots(GArgs a) {
  __shared__ double red[4 * 8 * 64];
  const int64_t total = a.N * a.ns;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double d[K];
#pragma unroll
  for (int q = 0; q < K; ++q) d[q] = 0.0;
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = (int)(e0 % a.ns);
  const double sc = a.inv[s];
  const int j = a.j, jl = j > 0 ? j - 1 : 0;  // last stored vector (v_0 when j = 0)
  double* Vj = a.V + (int64_t)j * total;
  for (int64_t e = e0; e < total; e += stride) {
    const int64_t pt = e / a.ns;
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = a.V[(int64_t)min(q, jl) * total + e];
    const double vj = a.W[e] * sc;
    const double w = gstencil(a.op, a.W, pt, a.ns, s) * sc;
    Vj[e] = vj;  // after the loads: with j = 0 they read this slot (and discard it)
    a.Wt[e] = w;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      // rows i < j from the basis, row j from the value just formed
      const double vq = q == j ? vj : v[q];
      d[q] = q <= j ? fma(vq, w, d[q]) : d[q];
    }
  }
  block_partials<K>(d, j + 1, a.ns, a.part, red);
}

// Update w -= sum_i hco[i] v_i; then either dots <v_i, w> (mode 0) or the
// squared norm (mode 1, written as row 0 of the partials).
template <int K>
__global__ __launch_bounds__(256) void g_update(GArgs a, int mode, double* out) {
  __shared__ double red[4 * 8 * 64];
  const int64_t total = a.N * a.ns;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double d[K], hc[K];
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = (int)(e0 % a.ns);  // fixed over the loop: ns divides the stride
  const int j = a.j;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    d[q] = 0.0;
    hc[q] = q <= j ? a.hco[q * a.ns + s] : 0.0;
  }
  for (int64_t e = e0; e < total; e += stride) {
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = a.V[(int64_t)min(q, j) * total + e];
    double w = a.Wt[e];
#pragma unroll
    for (int q = 0; q < K; ++q) w = fma(-hc[q], v[q], w);  // hc = 0 past row j
    out[e] = w;
    if (mode == 0) {
#pragma unroll
      for (int q = 0; q < K; ++q) d[q] = q <= j ? fma(v[q], w, d[q]) : d[q];
    } else {
      d[0] = fma(w, w, d[0]);
    }
  }
  block_partials<K>(d, mode == 0 ? j + 1 : 1, a.ns, a.part, red);
}

// Launches one pass with the smallest K that holds rows 0..j.
template <typename F>
static void with_k(int j, F&& f) {
  if (j + 1 <= 4) f(std::integral_constant<int, 4>());
  else if (j + 1 <= 8) f(std::integral_constant<int, 8>());
  else if (j + 1 <= 16) f(std::integral_constant<int, 16>());
  else if (j + 1 <= 32) f(std::integral_constant<int, 32>());
  else f(std::integral_constant<int, kMaxKrylov + 1>());
}

// h[q][s] = sum over workgroups of part[g][q][s]   (grid: (cnt, ns))
__global__ __launch_bounds__(256) void g_reduce(const double* part, int G, int K, int ns,
                                                double* h) {
  const int q = blockIdx.x, s = blockIdx.y;
  __shared__ double red[4];
  double t = 0.0;
  for (int g = threadIdx.x; g < G; g += 256) t += part[((int64_t)g * K + q) * ns + s];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) h[q * ns + s] = red[0] + red[1] + red[2] + red[3];
}

// Column j of H from the two passes and the norm; next scale 1/h_{j+1,j}.
__global__ void g_finish_column(const double* h1, const double* h2, const double* hn2,
                                double* H, double* inv, int m, int ns, int j) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  double* Hs = H + (int64_t)s * (m + 1) * m;
  double hs = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double v = h1[i * ns + s] + h2[i * ns + s];
    Hs[i * m + j] = v;
    hs = fma(v, v, hs);
  }
  const double hn = sqrt(fmax(hn2[s], 0.0));
  Hs[(j + 1) * m + j] = hn;
  // an (almost) invariant subspace contributes zero vectors from here on
  inv[s] = (hn > 1e-14 * sqrt(hs + hn * hn)) ? 1.0 / hn : 0.0;
}

__global__ void g_beta(const double* nrm2, double* beta, double* inv, int ns) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const double b = sqrt(fmax(nrm2[s], 0.0));
  beta[s] = b;
  inv[s] = b > 0.0 ? 1.0 / b : 0.0;
}

// exp(H_m) e_1 per state and Saad's estimate (relative to beta).
__global__ __launch_bounds__(256) void g_expm(const double* H, int m, double* f,
                                              double* est, double* estmax) {
  extern __shared__ double smem[];
  const int s = blockIdx.x;
  const double* Hs = H + (int64_t)s * (m + 1) * m;
  double* EA = smem;
  double* EW = EA + m * m;
  double* ER = EW + 5 * m * m;
  double* piv = ER + m * m;
  for (int idx = threadIdx.x; idx < m * m; idx += 256) EA[idx] = Hs[idx];
  __syncthreads();
  expm_small<256>(EA, m, EW, ER, piv);
  for (int i = threadIdx.x; i < m; i += 256) f[(int64_t)s * m + i] = ER[i * m];
  if (threadIdx.x == 0) {
    const double e = Hs[m * m + (m - 1)] * fabs(ER[(m - 1) * m]);
    est[s] = e;
    estmax[s] += e;
  }
}

// y = beta * sum_i f_i v_i
__global__ __launch_bounds__(256) void g_combine(const double* V, const double* f,
                                                 const double* beta, double* y,
                                                 int64_t total, int m, int ns) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += stride) {
    const int s = (int)(e % ns);
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc = fma(f[(int64_t)s * m + i], V[(int64_t)i * total + e], acc);
    y[e] = beta[s] * acc;
  }
}

// squared norms per state of x  -> part rows, reduced by g_reduce
template <int K>
__global__ __launch_bounds__(256) void g_norm(const double* x, int64_t total, int ns,
                                              double* part) {
  __shared__ double red[4 * 8 * 64];
  double d[K];
#pragma unroll
  for (int q = 0; q < K; ++q) d[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += stride)
    d[0] = fma(x[e], x[e], d[0]);
  block_partials<K>(d, 1, ns, part, red);
}

__global__ void g_check(const double* est, int ns, double tol, int* status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  if (!(est[s] <= tol)) atomicOr(status, est[s] != est[s] ? kStatusNonFinite : kStatusNotConverged);
}

// ----------------------------------------------------------------- driver --

int global_grid(int64_t total, int ns) {
  int64_t g = (total + 255) / 256;
  if (g > 1024) g = 1024;  // 4 workgroups per CU: each thread takes several points per reduction
  if (g < 1) g = 1;
  (void)ns;  // ns divides 256, so any grid keeps each thread on one state
  return (int)g;
}

size_t global_part_doubles(int G, int ns) { return (size_t)G * (kMaxKrylov + 1) * ns; }

// One global step (nsub sub-steps of Arnoldi of dimension m) on x -> y.
// Work: V ((m+1) N ns), W, Wt (N ns each), part, h1, h2, hn (small),
// H (ns (m+1) m), f (ns m), beta, inv, est (ns).
static void fill_op(const GlobalWork& w, GlobalOp& o, bool forced) {
  o.w0 = w.w[0]; o.wW = w.w[1]; o.wE = w.w[2]; o.wS = w.w[3]; o.wN = w.w[4];
  o.chx = w.chx; o.chy = w.chy; o.sub_scale = w.sub_scale;
  o.mux = w.mux; o.muy = w.muy; o.ax = w.ax; o.ay = w.ay; o.n = w.n; o.ndim = w.ndim;
  o.aug = forced ? 1 : 0;
  o.Npts = w.N;
  o.gscale = w.gscale;
  o.force = w.force;
}

// The three passes of Arnoldi column j and their reductions (partials are
// laid out with row stride K of the pass).
static void column_passes(GArgs& a, int G, int j, const GlobalWork& w, hipStream_t st) {
  with_k(j, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(g_spmv_dots<K>, dim3(G), dim3(256), 0, st, a);
    hipLaunchKernelGGL(g_reduce, dim3(j + 1, w.ns), dim3(256), 0, st, w.part, G, K, w.ns, w.h1);
    a.hco = w.h1;
    hipLaunchKernelGGL(g_update<K>, dim3(G), dim3(256), 0, st, a, 0, w.Wt);
    hipLaunchKernelGGL(g_reduce, dim3(j + 1, w.ns), dim3(256), 0, st, w.part, G, K, w.ns, w.h2);
    a.hco = w.h2;
    hipLaunchKernelGGL(g_update<K>, dim3(G), dim3(256), 0, st, a, 1, w.W);
    hipLaunchKernelGGL(g_reduce, dim3(1, w.ns), dim3(256), 0, st, w.part, G, K, w.ns, w.hn);
  });
}

hipError_t global_step(const GlobalWork& w, const double* x, double* y_out, hipStream_t st) {
  const bool forced = w.force != nullptr;
  const int64_t Na = w.N + (forced ? 1 : 0);  // points (plus the augmented coordinate)
  const int64_t total = Na * w.ns;
  const int G = global_grid(total, w.ns);
  const int m = w.m;
  GArgs a;
  fill_op(w, a.op, forced);
  a.V = w.V; a.W = w.W; a.Wt = w.Wt; a.part = w.part; a.N = Na; a.ns = w.ns;
  double* y = y_out;
  if (forced) {  // work on [x; 1]
    hipLaunchKernelGGL(g_aug_in, dim3(G), dim3(256), 0, st, x, w.xa, w.N * w.ns, w.ns);
    x = w.xa;
    y = w.ya;
  }
  const size_t lds = (size_t)(7 * m * m + 16) * 8;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)g_expm,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(g_zero_kernel, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.estsum,
                     (int64_t)w.ns);
  for (int sub = 0; sub < w.nsub; ++sub) {
    const double* src = sub == 0 ? x : y;
    zero_h(w, st);
    // beta = ||src||, W = src
    hipLaunchKernelGGL(g_norm<1>, dim3(G), dim3(256), 0, st, src, total, w.ns, w.part);
    hipLaunchKernelGGL(g_reduce, dim3(1, w.ns), dim3(256), 0, st, w.part, G, 1, w.ns, w.hn);
    hipLaunchKernelGGL(g_beta, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.hn, w.beta, w.inv, w.ns);
    a.W = const_cast<double*>(src);
    for (int j = 0; j < m; ++j) {
      a.j = j;
      a.inv = w.inv;
      column_passes(a, G, j, w, st);
      hipLaunchKernelGGL(g_finish_column, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.h1,
                         w.h2, w.hn, w.H, w.inv, m, w.ns, j);
      a.W = w.W;
    }
    hipLaunchKernelGGL(g_expm, dim3(w.ns), dim3(256), lds, st, w.H, m, w.f, w.est, w.estsum);
    hipLaunchKernelGGL(g_combine, dim3(G), dim3(256), 0, st, w.V, w.f, w.beta, y, total, m, w.ns);
  }
  hipLaunchKernelGGL(g_check, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.estsum, w.ns, w.tol,
                     w.status);
  if (forced) hipLaunchKernelGGL(g_copy, dim3(G), dim3(256), 0, st, y, y_out, w.N * w.ns);
  return hipGetLastError();
}

// Arnoldi only (dimension w.m, one sub-step) on x, exporting beta and H per
// state into calib (2 + (m+1) m doubles per state), for calibration.
hipError_t global_arnoldi(const GlobalWork& w, const double* x, double* calib, hipStream_t st) {
  const int64_t total = w.N * w.ns;
  const int G = global_grid(total, w.ns);
  const int m = w.m;
  GArgs a;
  fill_op(w, a.op, false);  // calibration runs on the unforced operator
  a.V = w.V; a.W = const_cast<double*>(x); a.Wt = w.Wt; a.part = w.part; a.N = w.N; a.ns = w.ns;
  zero_h(w, st);
  hipLaunchKernelGGL(g_norm<1>, dim3(G), dim3(256), 0, st, x, total, w.ns, w.part);
  hipLaunchKernelGGL(g_reduce, dim3(1, w.ns), dim3(256), 0, st, w.part, G, 1, w.ns, w.hn);
  hipLaunchKernelGGL(g_beta, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.hn, w.beta, w.inv, w.ns);
  for (int j = 0; j < m; ++j) {
    a.j = j;
    a.inv = w.inv;
    column_passes(a, G, j, w, st);
    hipLaunchKernelGGL(g_finish_column, dim3((w.ns + 255) / 256), dim3(256), 0, st, w.h1, w.h2,
                       w.hn, w.H, w.inv, m, w.ns, j);
    a.W = w.W;
  }
  hipLaunchKernelGGL(g_export_kernel, dim3(w.ns), dim3(256), 0, st, w.H, w.beta, m, calib);
  return hipGetLastError();
}

}  // namespace lem
