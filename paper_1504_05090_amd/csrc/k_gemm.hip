// Batched MFMA GEMM for gfx950 (FP32 and FP64 on 16x16x4 matrix cores).
//
// Used by the wraps G <- e^{-dtau K} (D G D^{-1}) e^{+dtau K}, the FP64 block
// products of the B chain and the UDV / fresh-G products.  A workgroup of 4
// wavefronts computes a BM x BN output tile; wavefront (wr, wc) owns a
// WM x WN quadrant of (WM/16) x (WN/16) MFMA blocks.  K advances in chunks of
// BK through a double-buffered LDS stage: the next chunk is fetched from
// global memory into registers while the current one feeds the MFMAs, so a
// chunk costs one barrier.  Optional diagonal
// scalings (of A's columns, of the result's rows and columns) are fused into
// the A fetch and the epilogue.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {

// LDS layouts.  An operand whose global rows run along k (A not transposed,
// B transposed) is staged k-contiguous, [m or n][BK + KP], and one whose rows
// run along m / n is staged [BK][BM or BN + 16]; either way a fetch writes
// consecutive words from consecutive lanes.  The pads make the MFMA operand
// reads (16 lanes along m or n times 4 lanes along k) hit distinct banks:
// KP = 4 words for FP32 and 2 doubles for FP64 spread the 16 rows of a
// k-contiguous tile over all banks; 16 elements shift the 4 k-rows of an
// m-contiguous tile by a quarter (FP32) or a half (FP64) of the 64 banks.
// largest K whose column scale is staged whole in LDS: the library's largest
// N for the big tiles, and 256 for the small ones (used below N = 192)
template <int BM, int BN> constexpr int gemm_ks_max() { return (BM >= 128 || BN >= 128) ? 512 : 256; }

template <typename T, bool TA, bool TB, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc d) {
  constexpr int WM = BM / 2, WN = BN / 2;          // 2 x 2 wavefronts
  constexpr int TM = WM / 16, TN = WN / 16;        // MFMA blocks per wavefront
  constexpr int KP = sizeof(T) == 4 ? 4 : 2;
  constexpr int A_ROWS = TA ? BK : BM, A_LD = TA ? BM + 16 : BK + KP;
  constexpr int B_ROWS = TB ? BN : BK, B_LD = TB ? BK + KP : BN + 16;
  constexpr int EA = BM * BK / 256, EB = BK * BN / 256;   // elements per thread per chunk
  __shared__ T As[2][A_ROWS][A_LD];
  __shared__ T Bs[2][B_ROWS][B_LD];
  __shared__ T Ksh[gemm_ks_max<BM, BN>()];   // A's column scale, staged once
  // the tile's row and column scales, staged for the big tiles (the small
  // ones would lose a workgroup per CU to the extra LDS)
  constexpr bool STAGE = BM >= 128;
  __shared__ T Rsh[STAGE ? BM : 1], Csh[STAGE ? BN : 1];

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
  const int l16 = lane & 15, lq = lane >> 4;

  // chunk element e of this thread -> (row, k) of A / (k, col) of B, chosen so
  // that consecutive threads read consecutive global addresses
  auto a_index = [&](int e, int &ii, int &kk) {
    const int idx = e * 256 + t;
    if (!TA) { ii = idx / BK; kk = idx % BK; } else { kk = idx / BM; ii = idx % BM; }
  };
  auto b_index = [&](int e, int &kk, int &jj) {
    const int idx = e * 256 + t;
    if (!TB) { kk = idx / BN; jj = idx % BN; } else { jj = idx / BK; kk = idx % BK; }
  };
  auto a_lds = [&](int buf, int ii, int kk) -> T & { return TA ? As[buf][kk][ii] : As[buf][ii][kk]; };
  auto b_lds = [&](int buf, int kk, int jj) -> T & { return TB ? Bs[buf][jj][kk] : Bs[buf][kk][jj]; };
  // A's column scale (staged in LDS once) is applied when a chunk is
  // stashed, so no fetched value is consumed before the current chunk's MFMAs
  T ra[EA], rb[EB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int ii, kk;
      a_index(e, ii, kk);
      const int gi = i0 + ii, gk = k0 + kk;
      T v = 0;
      if (gi < d.M && gk < d.K) v = TA ? A[(long)gk * d.lda + gi] : A[(long)gi * d.lda + gk];
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int kk, jj;
      b_index(e, kk, jj);
      const int gj = j0 + jj, gk = k0 + kk;
      T v = 0;
      if (gj < d.N && gk < d.K) v = TB ? B[(long)gj * d.ldb + gk] : B[(long)gk * d.ldb + gj];
      rb[e] = v;
    }
  };
  auto stash = [&](int buf, int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int ii, kk;
      a_index(e, ii, kk);
      const int gk = k0 + kk;
      a_lds(buf, ii, kk) = (ks && gk < d.K) ? ra[e] * Ksh[gk] : ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int kk, jj;
      b_index(e, kk, jj);
      b_lds(buf, kk, jj) = rb[e];
    }
  };

  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = acc_t{0, 0, 0, 0};

  const int nk = (d.K + BK - 1) / BK;
  fetch(0);
  // the epilogue's scales are staged while the first chunk loads, and read
  // after the main loop's barriers
  if (STAGE && rs)
    for (int e = t; e < BM; e += 256) Rsh[e] = i0 + e < d.M ? rs[i0 + e] : (T)0;
  if (STAGE && cs)
    for (int e = t; e < BN; e += 256) Csh[e] = j0 + e < d.N ? cs[j0 + e] : (T)0;
  if (ks) {
    for (int e = t; e < d.K; e += 256) Ksh[e] = ks[e];
    __syncthreads();
  }
  stash(0, 0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) fetch((kc + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = a_lds(buf, wr * WM + a * 16 + l16, kk + lq);
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = b_lds(buf, kk + lq, wc * WN + c * 16 + l16);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = Mfma<T>::mac(av[a], bv[c], acc[a][c]);
    }
    if (kc + 1 < nk) stash(buf ^ 1, (kc + 1) * BK);
    __syncthreads();
  }

  const T alpha = (T)d.alpha, beta = (T)d.beta;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wr * WM + a * 16 + Mfma<T>::row(lane, r);
        const int col = j0 + wc * WN + c * 16 + l16;
        if (row < d.M && col < d.N) {
          T v = alpha * acc[a][c][r];
          if (rs) v *= STAGE ? Rsh[row - i0] : rs[row];
          if (cs) v *= STAGE ? Csh[col - j0] : cs[col];
          T *dst = C + (long)row * d.ldc + col;
          if (beta != (T)0) v += beta * *dst;
          *dst = v;
        }
      }
}

template <typename T, int BM, int BN, int BK>
hipError_t launch_shape(const GemmDesc &d, bool ta, bool tb, hipStream_t s) {
  if (d.ks && d.K > gemm_ks_max<BM, BN>()) return hipErrorInvalidValue;
  const int tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  dim3 grid(tiles, d.batch), block(256);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<T, false, false, BM, BN, BK>), grid, block, 0, s, d);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm<T, true, false, BM, BN, BK>), grid, block, 0, s, d);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm<T, false, true, BM, BN, BK>), grid, block, 0, s, d);
  else hipLaunchKernelGGL((k_gemm<T, true, true, BM, BN, BK>), grid, block, 0, s, d);
  return hipSuccess;
}

template <typename T>
hipError_t launch(const GemmDesc &d, bool ta, bool tb, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.batch > 65535) return hipErrorInvalidValue;
  // tile shapes measured on the batched 256^3 products: FP32 128 x 256 with
  // 16-deep K chunks, FP64 128 x 128 with 8-deep chunks
  const bool big = d.M >= 192 && d.N >= 192;
  hipError_t e;
  if constexpr (sizeof(T) == 4) {
    e = big ? launch_shape<T, 128, 256, 16>(d, ta, tb, s) : launch_shape<T, 64, 64, 32>(d, ta, tb, s);
  } else {
    e = big ? launch_shape<T, 128, 128, 8>(d, ta, tb, s) : launch_shape<T, 64, 64, 16>(d, ta, tb, s);
  }
  return e != hipSuccess ? e : hipGetLastError();
}
}  // namespace

hipError_t gemm_f64(const GemmDesc &d, bool ta, bool tb, hipStream_t s) { return launch<double>(d, ta, tb, s); }
hipError_t gemm_f32(const GemmDesc &d, bool ta, bool tb, hipStream_t s) { return launch<float>(d, ta, tb, s); }

}  // namespace bss
