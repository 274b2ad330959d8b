// FP64 stabilisation kernels around the factorisations of k_qr.hip: the
// scale-separated fresh-G system and its right-hand side, the right-hand side
// of the time-displaced G, the drift/replace step and precision conversions.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {
// M = Db_R^{-1} (U_R^T U_L) Db_L^{-1} + Ds_R (V_R V_L^T) Ds_L   (W1 in, M out)
// or, without a left factor,  M = Db_R^{-1} U_R^T + Ds_R V_R;
// RHS = Db_R^{-1} U_R^T.
// One 32 x 32 tile of one matrix per workgroup (32 x 8 threads): the tile
// of U_R^T is staged through LDS so that both its read and the outputs are
// coalesced.
__global__ __launch_bounds__(256) void k_fresh_prep(const double *UR, const double *DR, const double *VR,
                                                    double *W1, const double *W2, const double *DL, double *RHS,
                                                    int N) {
  __shared__ double tile[32][33];
  const long NN = (long)N * N, m = blockIdx.y;
  const int tn = (N + 31) / 32, i0 = (blockIdx.x / tn) * 32, j0 = (blockIdx.x % tn) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {   // rows j0 + r of U_R, columns i0 + tx
    const int jj = j0 + r, ii = i0 + tx;
    tile[r][tx] = (jj < N && ii < N) ? UR[m * NN + (long)jj * N + ii] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i >= N || j >= N) continue;
    const long e = m * NN + (long)i * N + j;
    const double dr = DR[m * N + i];
    const double drb = big_part(dr), drs = dr / drb;
    const double ut = tile[tx][r] / drb;   // (U_R^T)_ij = U_R[j][i]
    RHS[e] = ut;
    if (DL) {
      const double dl = DL[m * N + j];
      const double dlb = big_part(dl), dls = dl / dlb;
      W1[e] = W1[e] / (drb * dlb) + drs * W2[e] * dls;
    } else {
      W1[e] = ut + drs * VR[e];
    }
  }
}

__global__ void k_time_rhs(const double *DR, const double *VR, double *RHS, int mats, int N) {
  const long NN = (long)N * N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN * mats) return;
  const long m = e / NN, r = e % NN;
  const double dr = DR[m * N + r / N];
  RHS[e] = (dr / big_part(dr)) * VR[e];
}

// drift = max_ij |G_cmp - G_fresh| over both spins of one chain, then the
// fresh matrices are written to G_out (rounded to its type).  G_cmp and G_out
// may be the same buffer.  Workgroup (p, c) takes part p of chain c and
// leaves its maxima of |G_cmp - G_fresh|, |G_fresh| and of the non-finite
// flag in part[c][p][0..2]; k_drift_final reduces them per chain.
template <typename Tc, typename To>
__global__ __launch_bounds__(256) void k_drift_part(const Tc *Gc, To *Go, const double *Gf, int N, double *part) {
  __shared__ double red[16];
  const long n = 2L * N * N, c = blockIdx.y;
  const long len = (n + DRIFT_PARTS - 1) / DRIFT_PARTS, e0 = blockIdx.x * len, e1 = min(n, e0 + len);
  const Tc *gc = Gc + c * n;
  To *go = Go + c * n;
  const double *gf = Gf + c * n;
  double dmax = 0.0, gmax = 0.0;
  bool bad = false;
  for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const double f = gf[e], g = (double)gc[e];
    // a non-finite fresh or wrapped G is a numerical failure (fmax would
    // drop a NaN difference)
    if (!isfinite(f) || !isfinite(g)) bad = true;
    dmax = fmax(dmax, fabs(g - f));
    gmax = fmax(gmax, fabs(f));
    go[e] = (To)f;
  }
  const double dm = block_max(dmax, red);
  const double gm = block_max(gmax, red);
  const double anybad = block_max(bad ? 1.0 : 0.0, red);
  if (threadIdx.x == 0) {
    double *pp = part + (c * DRIFT_PARTS + blockIdx.x) * 3;
    pp[0] = dm;
    pp[1] = gm;
    pp[2] = anybad;
  }
}

__global__ __launch_bounds__(64) void k_drift_final(const double *part, ChainStats *stats, int *err,
                                                    double drift_abort, int count) {
  const int c = blockIdx.x, p = threadIdx.x;
  const double *pp = part + ((long)c * DRIFT_PARTS + p) * 3;
  const double dm = wave_max(p < DRIFT_PARTS ? pp[0] : 0.0);
  const double gm = wave_max(p < DRIFT_PARTS ? pp[1] : 0.0);
  const double anybad = wave_max(p < DRIFT_PARTS ? pp[2] : 0.0);
  if (p == 0) {
    if (count) {
      ChainStats *st = stats + c;
      const double rel = dm / fmax(1.0, gm);
      st->drift_max = fmax(st->drift_max, dm);
      st->drift_sum += dm;
      st->rdrift_max = fmax(st->rdrift_max, rel);
      st->rdrift_sum += rel;
      st->rdrift_sweep = count == 2 ? rel : fmax(st->rdrift_sweep, rel);
      st->drift_count += 1;
      if (drift_abort > 0.0 && rel > drift_abort) atomicOr(err, 2);
    }
    if (anybad > 0.0) atomicOr(err, 4);
  }
}

template <typename Ts, typename Td>
__global__ void k_convert(const Ts *src, Td *dst, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (Td)src[e];
}
}  // namespace

hipError_t fresh_prep(const double *UR, const double *DR, const double *VR, double *W1, const double *W2,
                      const double *DL, double *RHS, int mats, int N, hipStream_t s) {
  if (mats <= 0) return hipSuccess;
  if (mats > 65535) return hipErrorInvalidValue;
  const int tn = (N + 31) / 32;
  hipLaunchKernelGGL(k_fresh_prep, dim3((unsigned)(tn * tn), (unsigned)mats), dim3(256), 0, s, UR, DR, VR, W1, W2,
                     DL, RHS, N);
  return hipGetLastError();
}

hipError_t time_rhs(const double *DR, const double *VR, double *RHS, int mats, int N, hipStream_t s) {
  const long n = (long)mats * N * N;
  hipLaunchKernelGGL(k_time_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, DR, VR, RHS, mats, N);
  return hipGetLastError();
}

hipError_t drift_replace(const void *Gc, bool cmp64, void *Go, bool out64, const double *Gf, int chains, int N,
                         double *part, ChainStats *stats, int *err, double drift_abort, int count, hipStream_t s) {
  if (chains <= 0) return hipSuccess;
  if (chains > 65535 || !part || count < 0 || count > 2) return hipErrorInvalidValue;
  const int cnt = count;
  const dim3 g(DRIFT_PARTS, chains), b(256);
  if (cmp64 && out64)
    hipLaunchKernelGGL((k_drift_part<double, double>), g, b, 0, s, (const double *)Gc, (double *)Go, Gf, N, part);
  else if (cmp64)
    hipLaunchKernelGGL((k_drift_part<double, float>), g, b, 0, s, (const double *)Gc, (float *)Go, Gf, N, part);
  else if (out64)
    hipLaunchKernelGGL((k_drift_part<float, double>), g, b, 0, s, (const float *)Gc, (double *)Go, Gf, N, part);
  else
    hipLaunchKernelGGL((k_drift_part<float, float>), g, b, 0, s, (const float *)Gc, (float *)Go, Gf, N, part);
  hipLaunchKernelGGL(k_drift_final, dim3(chains), dim3(64), 0, s, part, stats, err, drift_abort, cnt);
  return hipGetLastError();
}

hipError_t convert_green(const void *src, bool src64, void *dst, bool dst64, long n, hipStream_t s) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (src64 && !dst64)
    hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, s, (const double *)src, (float *)dst, n);
  else if (!src64 && dst64)
    hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, s, (const float *)src, (double *)dst, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace bss
