// Allocation-free global Krylov action: lem_global_expmv with every byte of
// device work space (status word, coefficients, Krylov basis, reduction
// partials, calibration probe) taken from one file-scope device array instead
// of hipMalloc.  The array is per device (each GPU the library runs on holds
// its own copy until the process ends); its address on the current device is
// looked up once with hipGetSymbolAddress and used for everything the host
// passes to kernels.  Calls that overlap on one device share the array and
// race; calls on different devices do not.
#include <hip/hip_runtime.h>

#include <mutex>

#include "arena.h"
#include "lem.h"
#include "lem_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// Device address of the scratch array on the current device.
lem_status scratch_base(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return lem::set_error(LEM_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices)
    return lem::set_error(LEM_ERR_UNSUPPORTED, "device index above the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return lem::set_error(LEM_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return LEM_OK;
}

}  // namespace

extern "C" lem_status lem_global_expmv_static(const lem_operator* op, double t, const double* x,
                                              double* y, int32_t n_states, double tol,
                                              int32_t m_max, void* stream) {
  if (!op) return lem::set_error(LEM_ERR_INVALID, "operator is NULL");
  if ((op->ndim != 1 && op->ndim != 2) || op->n < 3 || n_states < 1)
    return lem::set_error(LEM_ERR_INVALID, "bad operator size or n_states");
  if (lem::global_expmv_bound(op, n_states, m_max) > kScratchBytes)
    return lem::set_error(LEM_ERR_BUDGET,
                          "work space of this size exceeds the 64 MiB static scratch; use "
                          "lem_global_expmv");
  void* base = nullptr;
  const lem_status s = scratch_base(&base);
  if (s != LEM_OK) return s;
  lem::Arena arena((char*)base, kScratchBytes);
  return lem::global_expmv_in(op, t, x, y, n_states, tol, m_max, stream, &arena);
}
