// hawkes_grad_noalloc: the log-likelihood + gradient evaluation of hawkes_grad
// with its workspace in a library-owned static device array, for callers that
// cannot allocate device memory (graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/hawkes.h"
#include "hawkes_internal.hpp"

namespace hawkes {

// One static array per GPU (each device holds its own copy while the library
// is loaded).  Host code uses only the address hipGetSymbolAddress returns
// for the current device, never the array's name, which on the host is a
// stand-in, not a device address.
static __device__ __align__(256) unsigned char scratch[HAWKES_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// The current device's scratch address, looked up once per device with that
// device current (nullptr on a HIP error or a device ordinal out of range).
static void* scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace hawkes

extern "C" int hawkes_grad_noalloc(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p,
                                   int prec, void* stream, double* loglik, double* grad_x, double* grad_params) {
  if (!x || !t || !p || !grad_x) return HAWKES_EINVAL;
  const size_t need = hawkes_workspace_bytes(n, d, prec);
  if (need == 0) return HAWKES_EINVAL;
  if (need > HAWKES_NOALLOC_SCRATCH_BYTES) return HAWKES_ENOMEM;
  void* ws = hawkes::scratch_for_current_device();
  if (!ws) return HAWKES_EDEVICE;
  // every part of the workspace a call reads is written earlier in the same
  // call (the status words are cleared by its first kernel), so the previous
  // call's contents need no clearing
  hawkes::set_no_create(true);
  const int st = hawkes::run_sync(x, t, n, d, p, prec, ws, HAWKES_NOALLOC_SCRATCH_BYTES, stream, loglik, grad_x,
                                  grad_params);
  hawkes::set_no_create(false);
  return st;
}
