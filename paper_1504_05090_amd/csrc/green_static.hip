// Allocation-free variant of bss_green_from_field: its scratch is a
// file-scope device array of fixed size instead of a hipMalloc per call, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// Each device the library runs on holds its own copy of the array from the
// first call on it until the process ends.  Host code never uses the array's
// name as an address (on the host it is only a stand-in for the symbol): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept.  All calls on one device share the array, so calls that overlap on
// one device (different streams or host threads) race; calls in order on one
// stream are safe.  The recomputation writes every scratch value before
// reading it, so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bssqmc.h"
#include "green.h"

namespace {

// 12 MiB: one 16 x 16 field (N = 256) needs about 9.6 MB at n_stab = 8
constexpr size_t SCRATCH_BYTES = size_t(12) << 20;
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_dev[MAX_DEVICES];   // device address of `scratch`, per device

// the current device's address of the scratch array (looked up once, with
// that device current)
hipError_t scratch_address(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = static_cast<double *>(p);
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t bss_green_from_field_noalloc_limit(void) { return SCRATCH_BYTES; }

bss_status bss_green_from_field_noalloc(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab,
                                        int32_t l, const int8_t *field, double *G_out, void *stream) {
  size_t bytes = 0;
  const bss_status st = bss::green_check(L, U, t, beta, dtau, n_stab, l, field, G_out, &bytes);
  if (st != BSS_OK) return st;
  if (bytes > SCRATCH_BYTES) return BSS_E_UNSUPPORTED;
  double *base = nullptr;
  if (scratch_address(&base) != hipSuccess) return BSS_E_DEVICE;
  const hipError_t e = bss::green_run(L, U, t, beta, dtau, n_stab, l, field, G_out, base, (hipStream_t)stream);
  return e == hipSuccess ? BSS_OK : BSS_E_DEVICE;
}

}  // extern "C"
