// Products with the kinetic exponentials e^{-+dtau K} through their
// Kronecker factors.
//
// The hopping of eq. (1) on the periodic L x L square lattice is the sum of
// two commuting ring adjacencies (along x and along y), so
//   e^{-s K} = R (x) R,   R_{x x'} = r((x - x') mod L),
// with r the one-dimensional ring propagator.  With site i = x + L y, a
// product with it is two L-point circulant products per matrix column (left
// action) or row (right action): 4 L^5 multiply-adds per N x N matrix
// (N = L^2) in place of the 2 L^6 of a dense product -- the same matrix up to
// rounding.  The kernels are bound by HBM traffic: every element of X is read
// once and every element of Y written once.
//
// Left action  Y = (R (x) R) diag(ks) X, one workgroup per strip of W
//   columns: the strip (all N rows) is staged in LDS, then the x-mode products
//   run per (column, y) in place and the y-mode products per (column, x) go
//   straight to Y.
// Right action Y = diag(rs) X diag(ks) (R (x) R), one workgroup per strip of
//   RW rows: the same two passes along each row's (y, x) index.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {

constexpr int HOP_THREADS = 256;

// columns per left-action strip: rows of W elements span a 128-byte line
// (FP64 16, FP32 32) where the LDS strip fits 64 KB, half of that above
template <typename T, int L> constexpr int strip_cols() {
  return (sizeof(T) == 8 ? 16 : 32) / (L > 16 ? 2 : 1);
}
// rows per right-action strip
template <int L> constexpr int strip_rows() { return L > 16 ? 8 : 16; }

template <typename T, int L>
__global__ __launch_bounds__(HOP_THREADS) void k_hop_left(HopDesc d) {
  constexpr int N = L * L, W = strip_cols<T, L>(), LD = W + 1;
  constexpr int CNT = (N * W + HOP_THREADS - 1) / HOP_THREADS;
  __shared__ T S[N * LD];
  const int t = threadIdx.x;
  const long m = blockIdx.y;
  const int j0 = blockIdx.x * W;
  const T *X = (const T *)d.X + m * d.sX;
  T *Y = (T *)d.Y + m * d.sY;
  const T *ks = d.ks ? (const T *)d.ks + m * d.sks : nullptr;
  T c[L];
#pragma unroll
  for (int q = 0; q < L; ++q) c[q] = ((const T *)d.r)[q];

  // stage the strip: consecutive threads read consecutive columns of a row
  T v[CNT];
#pragma unroll
  for (int q = 0; q < CNT; ++q) {
    const int e = q * HOP_THREADS + t, i = e / W, j = e % W;
    T x = 0;
    if (e < N * W && j0 + j < N) {
      x = X[(long)i * N + j0 + j];
      if (ks) x *= ks[i];
    }
    v[q] = x;
  }
#pragma unroll
  for (int q = 0; q < CNT; ++q) {
    const int e = q * HOP_THREADS + t;
    if (e < N * W) S[(e / W) * LD + e % W] = v[q];
  }
  __syncthreads();

  // x-mode: Z[(x, y)] = sum_x' r(x - x') X[(x', y)], in place per (column, y)
  for (int task = t; task < W * L; task += HOP_THREADS) {
    const int j = task % W, y = task / W;
    T a[L];
#pragma unroll
    for (int x = 0; x < L; ++x) a[x] = S[(y * L + x) * LD + j];
#pragma unroll
    for (int x = 0; x < L; ++x) {
      T s = 0;
#pragma unroll
      for (int xp = 0; xp < L; ++xp) s += c[(x - xp + L) % L] * a[xp];
      S[(y * L + x) * LD + j] = s;
    }
  }
  __syncthreads();

  // y-mode: Y[(x, y)] = sum_y' r(y - y') Z[(x, y')], per (column, x)
  for (int task = t; task < W * L; task += HOP_THREADS) {
    const int j = task % W, x = task / W;
    if (j0 + j >= N) continue;
    T a[L];
#pragma unroll
    for (int y = 0; y < L; ++y) a[y] = S[(y * L + x) * LD + j];
#pragma unroll
    for (int y = 0; y < L; ++y) {
      T s = 0;
#pragma unroll
      for (int yp = 0; yp < L; ++yp) s += c[(y - yp + L) % L] * a[yp];
      Y[(long)(y * L + x) * N + j0 + j] = s;
    }
  }
}

template <typename T, int L>
__global__ __launch_bounds__(HOP_THREADS) void k_hop_right(HopDesc d) {
  constexpr int N = L * L, RW = strip_rows<L>(), LP = L + 1, RS = L * LP;
  constexpr int CNT = (N * RW + HOP_THREADS - 1) / HOP_THREADS;
  __shared__ T S[RW * RS];
  const int t = threadIdx.x;
  const long m = blockIdx.y;
  const int i0 = blockIdx.x * RW;
  const T *X = (const T *)d.X + m * d.sX;
  T *Y = (T *)d.Y + m * d.sY;
  const T *ks = d.ks ? (const T *)d.ks + m * d.sks : nullptr;
  const T *rs = d.rs ? (const T *)d.rs + m * d.srs : nullptr;
  T c[L];
#pragma unroll
  for (int q = 0; q < L; ++q) c[q] = ((const T *)d.r)[q];

  // stage RW rows, each split into its (y, x) index with padded y stride
  T v[CNT];
#pragma unroll
  for (int q = 0; q < CNT; ++q) {
    const int e = q * HOP_THREADS + t, r = e / N, jj = e % N;
    T x = 0;
    if (e < N * RW && i0 + r < N) {
      x = X[(long)(i0 + r) * N + jj];
      if (ks) x *= ks[jj];
      if (rs) x *= rs[i0 + r];
    }
    v[q] = x;
  }
#pragma unroll
  for (int q = 0; q < CNT; ++q) {
    const int e = q * HOP_THREADS + t, r = e / N, jj = e % N;
    if (e < N * RW) S[r * RS + (jj / L) * LP + jj % L] = v[q];
  }
  __syncthreads();

  // x-mode: Z[(x, y)] = sum_x' X[(x', y)] r(x' - x), in place per (row, y)
  for (int task = t; task < RW * L; task += HOP_THREADS) {
    const int y = task % L, r = task / L;
    T a[L];
#pragma unroll
    for (int x = 0; x < L; ++x) a[x] = S[r * RS + y * LP + x];
#pragma unroll
    for (int x = 0; x < L; ++x) {
      T s = 0;
#pragma unroll
      for (int xp = 0; xp < L; ++xp) s += a[xp] * c[(xp - x + L) % L];
      S[r * RS + y * LP + x] = s;
    }
  }
  __syncthreads();

  // y-mode: Y[(x, y)] = sum_y' Z[(x, y')] r(y' - y), per (row, x)
  for (int task = t; task < RW * L; task += HOP_THREADS) {
    const int x = task % L, r = task / L;
    if (i0 + r >= N) continue;
    T a[L];
#pragma unroll
    for (int y = 0; y < L; ++y) a[y] = S[r * RS + y * LP + x];
#pragma unroll
    for (int y = 0; y < L; ++y) {
      T s = 0;
#pragma unroll
      for (int yp = 0; yp < L; ++yp) s += a[yp] * c[(yp - y + L) % L];
      Y[(long)(i0 + r) * N + y * L + x] = s;
    }
  }
}

template <typename T, int L>
void launch_l(const HopDesc &d, bool left, hipStream_t s) {
  constexpr int N = L * L;
  if (left) {
    constexpr int W = strip_cols<T, L>();
    hipLaunchKernelGGL((k_hop_left<T, L>), dim3((N + W - 1) / W, d.mats), dim3(HOP_THREADS), 0, s, d);
  } else {
    constexpr int RW = strip_rows<L>();
    hipLaunchKernelGGL((k_hop_right<T, L>), dim3((N + RW - 1) / RW, d.mats), dim3(HOP_THREADS), 0, s, d);
  }
}

template <typename T>
hipError_t launch(const HopDesc &d, bool left, hipStream_t s) {
  if (d.mats <= 0) return hipSuccess;
  if (d.mats > 65535 || !d.X || !d.Y || !d.r || d.X == d.Y) return hipErrorInvalidValue;
  switch (d.L) {
    case 2: launch_l<T, 2>(d, left, s); break;
    case 4: launch_l<T, 4>(d, left, s); break;
    case 6: launch_l<T, 6>(d, left, s); break;
    case 8: launch_l<T, 8>(d, left, s); break;
    case 10: launch_l<T, 10>(d, left, s); break;
    case 12: launch_l<T, 12>(d, left, s); break;
    case 14: launch_l<T, 14>(d, left, s); break;
    case 16: launch_l<T, 16>(d, left, s); break;
    case 18: launch_l<T, 18>(d, left, s); break;
    case 20: launch_l<T, 20>(d, left, s); break;
    case 22: launch_l<T, 22>(d, left, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t hop_left(const HopDesc &d, bool f64, hipStream_t s) {
  return f64 ? launch<double>(d, true, s) : launch<float>(d, true, s);
}
hipError_t hop_right(const HopDesc &d, bool f64, hipStream_t s) {
  return f64 ? launch<double>(d, false, s) : launch<float>(d, false, s);
}

}  // namespace bss
