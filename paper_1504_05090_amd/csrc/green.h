// Recomputation of one field's equal-time Green functions (both spins) on a
// caller-given scratch region (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bssqmc.h"

namespace bss {

// Validates the arguments of bss_green_from_field; *scratch_bytes receives the
// device scratch the recomputation needs.
bss_status green_check(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                       const int8_t *field, const double *G_out, size_t *scratch_bytes);
// Enqueues the recomputation on s with its scratch at base (green_check's
// size, 256-byte aligned); every scratch value is written before it is read.
hipError_t green_run(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                     const int8_t *field, double *G_out, double *base, hipStream_t s);

}  // namespace bss
