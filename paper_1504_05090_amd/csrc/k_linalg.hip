// FP64 stabilisation kernels: pre-pivoted Householder QR for the UDV
// factorisation of the B chain (Loh & Gubernatis), the QR solve of the
// scale-separated fresh-G system, and the drift/replace step.
//
// One workgroup factors one matrix; the matrix lives in global memory (L2 /
// MALL resident) and the current Householder vector in LDS.  Pivoting is done
// once up front (columns sorted by decreasing norm, Bai, Lee, Li & Xu 2011),
// which orders the graded scales of X = P U D the way column pivoting would.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {
constexpr int QT = 256;      // threads per factorisation
constexpr int NMAX = 512;

// Householder reflector of column j of W (rows j..N-1): W[j:,j] -> alpha e_1.
// Leaves v in vcur[j..N-1] and returns tau; alpha in *alpha.
__device__ double householder_col(const double *W, int N, int j, double *vcur, double *red, double *alpha) {
  double part = 0.0;
  for (int r = j + threadIdx.x; r < N; r += blockDim.x) {
    const double x = W[(long)r * N + j];
    vcur[r] = x;
    part += x * x;
  }
  const double nrm2 = block_sum(part, red);
  const double x0 = vcur[j];
  const double a = x0 > 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
  const double v0 = x0 - a;
  const double vn2 = nrm2 - x0 * x0 + v0 * v0;
  __syncthreads();
  if (threadIdx.x == 0) vcur[j] = v0;
  __syncthreads();
  *alpha = a;
  return vn2 > 0.0 ? 2.0 / vn2 : 0.0;
}

// X (overwritten with the factor) -> U = Q, D = diag R, RP = D^{-1} R Pi^T.
__global__ __launch_bounds__(QT) void k_qr_udv(double *Xall, double *Uall, double *Dall, double *RPall, int N) {
  __shared__ double norms[NMAX], vcur[NMAX], vhead[NMAX], tau[NMAX], rdiag[NMAX];
  __shared__ int perm[NMAX];
  __shared__ double red[16];
  const long NN = (long)N * N, b = blockIdx.x;
  double *X = Xall + b * NN, *U = Uall + b * NN, *RP = RPall + b * NN, *D = Dall + b * N;
  double *W = RP;   // the permuted copy is factored in the RP buffer, RP written last
  const int t = threadIdx.x, nt = blockDim.x;

  for (int q = t; q < N; q += nt) {
    double s = 0.0;
    for (int r = 0; r < N; ++r) { const double x = X[(long)r * N + q]; s += x * x; }
    norms[q] = s;
  }
  __syncthreads();
  for (int q = t; q < N; q += nt) {
    int rank = 0;
    const double nq = norms[q];
    for (int p = 0; p < N; ++p) rank += (norms[p] > nq) || (norms[p] == nq && p < q);
    perm[rank] = q;
  }
  __syncthreads();
  for (long e = t; e < NN; e += nt) W[e] = X[(e / N) * N + perm[e % N]];
  __syncthreads();

  for (int j = 0; j < N; ++j) {
    double alpha;
    const double tj = householder_col(W, N, j, vcur, red, &alpha);
    if (t == 0) { tau[j] = tj; vhead[j] = vcur[j]; rdiag[j] = alpha; }
    if (tj != 0.0) {
      for (int q = j + 1 + t; q < N; q += nt) {
        double wq = 0.0;
        for (int r = j; r < N; ++r) wq += vcur[r] * W[(long)r * N + q];
        wq *= tj;
        for (int r = j; r < N; ++r) W[(long)r * N + q] -= wq * vcur[r];
      }
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{N-1}: apply the reflectors to I from the last one
  for (long e = t; e < NN; e += nt) U[e] = ((e / N) == (e % N)) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = N - 1; j >= 0; --j) {
    for (int r = j + 1 + t; r < N; r += nt) vcur[r] = W[(long)r * N + j];
    if (t == 0) vcur[j] = vhead[j];
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      for (int q = j + t; q < N; q += nt) {
        double wq = 0.0;
        for (int r = j; r < N; ++r) wq += vcur[r] * U[(long)r * N + q];
        wq *= tj;
        for (int r = j; r < N; ++r) U[(long)r * N + q] -= wq * vcur[r];
      }
    }
    __syncthreads();
  }
  // D and RP = D^{-1} R Pi^T:  RP[i][perm[q]] = R[i][q] / R[i][i]
  for (int i = t; i < N; i += nt) D[i] = rdiag[i];
  // X is free now: build RP there, then copy (W and RP share storage)
  for (long e = t; e < NN; e += nt) {
    const int i = (int)(e / N), q = (int)(e % N);
    const double v = q < i ? 0.0 : (q == i ? 1.0 : W[e] / rdiag[i]);
    X[(long)i * N + perm[q]] = v;
  }
  __syncthreads();
  for (long e = t; e < NN; e += nt) RP[e] = X[e];
}

// Solve M Z = B (N right-hand sides) by Householder QR of M.
__global__ __launch_bounds__(QT) void k_qr_solve(double *Mall, double *Ball, int N) {
  __shared__ double vcur[NMAX], rdiag[NMAX];
  __shared__ double red[16];
  const long NN = (long)N * N, b = blockIdx.x;
  double *M = Mall + b * NN, *B = Ball + b * NN;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < N; ++j) {
    double alpha;
    const double tj = householder_col(M, N, j, vcur, red, &alpha);
    if (t == 0) rdiag[j] = alpha;
    if (tj != 0.0) {
      // trailing columns of M (q > j) and every column of B
      for (int q = j + 1 + t; q < 2 * N; q += nt) {
        double *col = q < N ? M + q : B + (q - N);
        double wq = 0.0;
        for (int r = j; r < N; ++r) wq += vcur[r] * col[(long)r * N];
        wq *= tj;
        for (int r = j; r < N; ++r) col[(long)r * N] -= wq * vcur[r];
      }
    }
    __syncthreads();
  }
  // back substitution R Z = Q^T B, one column of B per thread
  for (int q = t; q < N; q += nt) {
    for (int i = N - 1; i >= 0; --i) {
      double s = B[(long)i * N + q];
      for (int c = i + 1; c < N; ++c) s -= M[(long)i * N + c] * B[(long)c * N + q];
      B[(long)i * N + q] = s / rdiag[i];
    }
  }
}

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

hipError_t qr_udv(double *X, double *U, double *D, double *RP, int mats, int N, hipStream_t s) {
  if (N > NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qr_udv, dim3(mats), dim3(QT), 0, s, X, U, D, RP, N);
  return hipGetLastError();
}

hipError_t qr_solve(double *M, double *B, int mats, int N, hipStream_t s) {
  if (N > NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qr_solve, dim3(mats), dim3(QT), 0, s, M, B, N);
  return hipGetLastError();
}

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
