// Order of columns for the pivoted QR (k_qr.hip): by decreasing squared norm,
// a NaN norm counting as -1 (below every norm, so it ranks last), equal keys
// by increasing index.  This is a strict total order on (key, index) pairs,
// so the ranks of n columns counted with it are a permutation of 0..n-1 and
// the pivot found by any reduction order is the same column.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace bss {

__host__ __device__ __forceinline__ double rank_key(double norm2) { return std::isnan(norm2) ? -1.0 : norm2; }

// column (a, ia) comes before column (b, ib); a and b are rank keys
__host__ __device__ __forceinline__ bool ranks_before(double a, int ia, double b, int ib) {
  return a > b || (a == b && ia < ib);
}

}  // namespace bss
