// Device measurement accumulators (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bss {

struct MeasState {
  double *docc;      // [chains][nbins]
  double *gk;        // [chains][nbins_g][glen], glen = (Lambda+1) N
  double *sc;        // [chains][nbins_g][sclen], sclen = N: spin correlation C(r)
  int64_t *count;    // [chains] measurements taken
  int64_t *binsize;  // [chains]
  int *cur;          // [chains] bin of the measurement in progress
  int nbins, nbins_g;
  long glen, sclen;
};

hipError_t meas_begin(const MeasState &ms, int chains, hipStream_t s);
hipError_t meas_end(const MeasState &ms, int chains, hipStream_t s);
hipError_t meas_docc(const MeasState &ms, const double *Gf, int chains, int N, hipStream_t s);
hipError_t meas_gk(const MeasState &ms, const double *Gt, int chains, int L, int l, hipStream_t s);
hipError_t meas_sc(const MeasState &ms, const double *Gf, int chains, int L, hipStream_t s);

}  // namespace bss
