// The projected product C = A *_Q B (Def. 3.1) for callers that cannot
// allocate device memory: the transform-domain intermediates Ahat, Bhat and
// Chat, which pq_qprod takes from its ws argument, live in a fixed array of
// this library's code object instead.  The kernels are pq_qprod's own; only
// where their scratch memory comes from differs.
//
// The array is a device symbol: the name `scratch` in host code is a
// host-side stand-in, not a device address.  The device address is asked of
// the runtime once per device, with that device current, and kept; every
// later use (the workspace pointer handed to the kernels) is that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/projprod.h"
#include "internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[PQ_QPROD_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// The device address of the current device's copy of the array, looked up on
// the first call on that device.
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int pq_qprod_noalloc(const void* A, const void* B, int ab_dtype, const void* Q, void* C, int64_t n1,
                                int64_t m, int64_t n2, int64_t n3, int64_t p, int prec, void* Ahat_out,
                                void* Bhat_out, hipStream_t stream) {
  if (!A || !B || !Q || !C) return PQ_ERR_NULL;
  if (ab_dtype != PQ_F32 && ab_dtype != PQ_F64 && ab_dtype != PQ_BF16) return PQ_ERR_DTYPE;
  if (n1 < 1 || m < 1 || n2 < 1 || n3 < 1) return PQ_ERR_SHAPE;
  if (p < 1 || p > n3) return PQ_ERR_P;
  // sizes whose intermediates exceed the array are refused before the
  // device is touched (each factor is checked first so that the byte count
  // cannot overflow)
  const int64_t lim = (int64_t)PQ_QPROD_NOALLOC_MAX_BYTES;
  if (n1 > lim || m > lim || n2 > lim || p > lim || n1 * m > lim || m * n2 > lim || n1 * n2 > lim)
    return PQ_ERR_UNSUPPORTED;
  const size_t need = pq_qprod_workspace(n1, m, n2, n3, p, ab_dtype);
  if (need > (size_t)PQ_QPROD_NOALLOC_MAX_BYTES) return PQ_ERR_UNSUPPORTED;
  void* ws = nullptr;
  const hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) return pq::note_hip_error(e);
  return pq_qprod(A, B, ab_dtype, Q, C, n1, m, n2, n3, p, prec, Ahat_out, Bhat_out, ws,
                  (size_t)PQ_QPROD_NOALLOC_MAX_BYTES, stream);
}
