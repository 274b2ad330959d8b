// Batched MFMA GEMM for gfx950 (FP32 and FP64, 16x16x4 matrix cores).
//
// Used by the wraps G <- e^{-dtau K} (D G D^{-1}) e^{+dtau K}, the FP64
// block products of the B chain and the UDV / fresh-G products.  One
// workgroup of 4 wavefronts computes a 64 x 64 output tile; each wavefront
// owns a 32 x 32 quadrant (2 x 2 MFMA blocks).  K is staged through LDS in
// chunks of 16.  Optional diagonal scalings (of A's columns, of the result's
// rows and columns) are fused into the tile loads and the epilogue.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {
constexpr int BM = 64, BN = 64, BK = 16;

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc d) {
  __shared__ T As[BM][BK + 1];
  __shared__ T Bs[BK][BN + 1];
  const int tilesN = (d.N + BN - 1) / BN;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
  const long b = blockIdx.y;
  const T *A = (const T *)d.A + b * d.sA;
  const T *B = (const T *)d.B + b * d.sB;
  T *C = (T *)d.C + b * d.sC;
  const T *ks = d.ks ? (const T *)d.ks + b * d.sks : nullptr;
  const T *rs = d.rs ? (const T *)d.rs + b * d.srs : nullptr;
  const T *cs = d.cs ? (const T *)d.cs + b * d.scs : nullptr;
  const int i0 = tm * BM, j0 = tn * BN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < d.K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t * 4 + e;
      int ii, kk;
      if (!TA) { ii = idx / BK; kk = idx % BK; } else { kk = idx / BM; ii = idx % BM; }
      const int gi = i0 + ii, gk = k0 + kk;
      T v = 0;
      if (gi < d.M && gk < d.K) {
        v = TA ? A[(long)gk * d.lda + gi] : A[(long)gi * d.lda + gk];
        if (ks) v *= ks[gk];
      }
      As[ii][kk] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t * 4 + e;
      int jj, kk;
      if (!TB) { kk = idx / BN; jj = idx % BN; } else { jj = idx / BK; kk = idx % BK; }
      const int gj = j0 + jj, gk = k0 + kk;
      T v = 0;
      if (gj < d.N && gk < d.K) v = TB ? B[(long)gj * d.ldb + gk] : B[(long)gk * d.ldb + gj];
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[wr * 32 + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = Bs[kk + (lane >> 4)][wc * 32 + c * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = Mfma<T>::mac(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
  const T alpha = (T)d.alpha, beta = (T)d.beta;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wr * 32 + a * 16 + Mfma<T>::row(lane, r);
        const int col = j0 + wc * 32 + c * 16 + (lane & 15);
        if (row < d.M && col < d.N) {
          T v = alpha * acc[a][c][r];
          if (rs) v *= rs[row];
          if (cs) v *= cs[col];
          T *dst = C + (long)row * d.ldc + col;
          if (beta != (T)0) v += beta * *dst;
          *dst = v;
        }
      }
}

template <typename T>
hipError_t launch(const GemmDesc &d, bool ta, bool tb, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.batch > 65535) return hipErrorInvalidValue;
  const int tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  dim3 grid(tiles, d.batch), block(256);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<T, false, false>), grid, block, 0, s, d);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm<T, true, false>), grid, block, 0, s, d);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm<T, false, true>), grid, block, 0, s, d);
  else hipLaunchKernelGGL((k_gemm<T, true, true>), grid, block, 0, s, d);
  return hipGetLastError();
}
}  // namespace

hipError_t gemm_f64(const GemmDesc &d, bool ta, bool tb, hipStream_t s) { return launch<double>(d, ta, tb, s); }
hipError_t gemm_f32(const GemmDesc &d, bool ta, bool tb, hipStream_t s) { return launch<float>(d, ta, tb, s); }

}  // namespace bss
