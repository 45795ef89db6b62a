// Local matrices of the 1D Schroedinger equation with a harmonic potential
// (section 4.1; gfx950):
//
//   c_t = (i/2) c_xx - i (kappa/2) x^2 c  on [-L/2, L/2), periodic,
//   c' = -i H c,   H = -(1/2) D2 + diag(kappa x_j^2 / 2)   (centered differences)
//
// The complex problem is carried by its real form: with c = a + i b,
// a' = H b and b' = -H a.  Unknowns are interleaved per node (a_j, b_j), so
// the state is a real vector of 2n entries and a region of nl nodes is a
// contiguous run of 2 nl of them; the local matrix dt [[0, H_M], [-H_M, 0]]
// (interleaved) is the real form of -i dt H_M, and its exponential is the
// real form of the complex local exponential.  The stored-block machinery of
// the dense method (Pade [13/13] on FP64 MFMA, packed core rows, the MFMA
// apply) then runs unchanged on the doubled grid.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lem_launch.h"

namespace lem {

struct SchBox {
  int ox, h, whole;  // first node of the region's buffer is ox - h (mod n)
};

__device__ __forceinline__ int sch_wrap(int a, int n) {
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// A[u] (m x m, m = 2 nl, row-major) = dt * real form of -i H on region u.
__global__ void sch_assemble_kernel(const SchBox* boxes, int nb, int nl, int n, double L,
                                    double kappa, double dt, double* A) {
  const int m = 2 * nl;
  const int64_t per = (int64_t)m * m, total = per * nb;
  const double dx = L / n, off = -0.5 / (dx * dx);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(e / per);
    const int64_t rc = e - (int64_t)u * per;
    const int r = (int)(rc / m), c = (int)(rc - (int64_t)r * m);
    const int lr = r >> 1, lc = c >> 1, pr = r & 1, pc = c & 1;
    double v = 0.0;
    if (pr != pc) {
      const SchBox b = boxes[u];
      double h = 0.0;  // H_M(lr, lc)
      if (lr == lc) {
        const double x = -0.5 * L + sch_wrap(b.ox - b.h + lr, n) * dx;
        h = 1.0 / (dx * dx) + 0.5 * kappa * x * x;
      } else if (lc == lr - 1 || lc == lr + 1 ||
                 (b.whole && ((lr == 0 && lc == nl - 1) || (lr == nl - 1 && lc == 0)))) {
        h = off;
      }
      v = (pr == 0 ? dt : -dt) * h;  // a' = H b, b' = -H a
    }
    A[e] = v;
  }
}

size_t sch_box_size() { return sizeof(SchBox); }

void sch_box_fill(void* dst, int i, int ox, int h, int whole) {
  SchBox* b = (SchBox*)dst + i;
  b->ox = ox; b->h = h; b->whole = whole;
}

hipError_t sch_assemble(const void* boxes, int nb, int nl, int n, double L, double kappa,
                        double dt, double* A, hipStream_t st) {
  const int64_t total = (int64_t)4 * nl * nl * nb;
  int64_t g = (total + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(sch_assemble_kernel, dim3((unsigned)(g < 1 ? 1 : g)), dim3(256), 0, st,
                     (const SchBox*)boxes, nb, nl, n, L, kappa, dt, A);
  return hipGetLastError();
}

}  // namespace lem
