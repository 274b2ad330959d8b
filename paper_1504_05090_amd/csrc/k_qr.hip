// Blocked Householder QR in FP64 for the UDV stabilisation (gfx950).
//
// One workgroup factors one matrix of the batch.  Columns are processed in
// panels of NB.  A panel is factored in LDS (unblocked Householder with
// wavefront reductions for the norms), its reflectors are aggregated into the
// compact WY form Q_p = I - V T V^T (Schreiber & Van Loan), and the trailing
// columns are updated chunk by chunk with two FP64 MFMA products,
//   W = V^T C,   C <- C - V (T^T W),
// the chunk C staying in registers in the MFMA accumulator layout.
//
// Pivoting for the UDV factorisation follows Businger-Golub: every pivot is
// the remaining column of largest norm.  Before each panel the remaining
// columns are ranked by their current norms (accumulated while the previous
// panel's update streams through them) and the NB largest are swapped into
// the panel, where the pivots are searched column by column.  A column's norm
// over the remaining rows never grows under the panel's reflections, so while
// the best in-panel norm is at least the largest norm left outside the panel
// (taken at the panel's start), the in-panel pivot is the global one.  When
// it falls below, the panel ends there and its unfactored columns go back to
// the trailing matrix: panels have variable width, and |R_ij| <= |R_ii| holds
// as it does for unblocked Businger-Golub pivoting.
//
//   qr_udv:   X Pi = Q R  ->  U = Q, D = diag R, RP = D^{-1} R Pi^T
//
// The file also holds the solve of the fresh-G system by blocked LU with
// partial pivoting (k_lu_solve), which shares the LDS layout and the blocked
// back substitution:
//   lu_solve: P M = L U,  Z = U^-1 L^-1 P B
#include "common.h"
#include "kernels.h"
#include "qr_order.h"

namespace bss {

namespace {

constexpr int QT = 256;   // 4 wavefronts
typedef Mfma<double> M64;


// per-shape constants: panel width NB, chunk width CW, max row tiles per wave;
// COLS: block reflectors applied by whole-column tiles per wavefront
// (apply_cols, every row of a tile in registers), else by row tiles
// (apply_block)
template <int NB_, int CW_, int RTW_, bool COLS_> struct Shape {
  static constexpr int NB = NB_, CW = CW_, RTW = RTW_;
  static constexpr bool COLS = COLS_;
  static constexpr int LDV = NB + 1;
  static constexpr int CT = CW / 16;   // column tiles per chunk
  static constexpr int WT = NB / 16;   // row tiles of W
  static constexpr int MT = 4 * RTW;   // row tiles of the largest matrix
};
typedef Shape<32, 64, 4, true> ShapeS;    // N <= 256
typedef Shape<16, 32, 8, false> ShapeL;   // N <= 512

struct Lds {
  double *V;      // [mr][LDV] panel / clean reflectors
  double *Wp;     // [4][NB][CW] per-wave partials of V^T C
  double *W2;     // [NB][CW]   -op(T) W
  double *T;      // [NB][NB]
  double *tau;    // [NB]
  double *beta;   // [NB]
  double *red;    // [64]
  double *pn;     // [NB] in-panel pivot norms (rows >= j)
  double *pg;     // [NB] (rows > j)
  double *norms;  // [N]  current column norms (udv)
  double *nuout;  // [1]  largest squared norm outside the panel at its start (udv)
  double *npart;  // [4][CW] per-wave partial norms (aliases the spare partials of Wp)
  int *orig;      // [N]  original index of each physical column (udv)
  int *sel;       // [N + 3 NB + 1] scratch for the panel selection
};

__device__ __forceinline__ int round16(int x) { return (x + 15) & ~15; }

template <class S>
__device__ Lds carve(char *base, int N) {
  Lds s;
  const int mr = round16(N);
  double *p = (double *)base;
  s.V = p; p += mr * S::LDV;
  s.Wp = p; p += 4 * S::NB * S::CW;
  s.W2 = p; p += S::NB * S::CW;
  s.T = p; p += S::NB * S::NB;
  s.tau = p; p += S::NB;
  s.beta = p; p += S::NB;
  s.red = p; p += 64;
  s.pn = p; p += S::NB;
  s.pg = p; p += S::NB;
  s.norms = p; p += N;
  s.nuout = p; p += 1;
  s.npart = s.Wp + S::NB * S::CW;   // partial 1..3 of Wp are free once W is summed
  s.orig = (int *)p;
  s.sel = s.orig + N;
  return s;
}

template <class S>
size_t lds_bytes(int N) {
  const int mr = (N + 15) & ~15;
  const size_t d = (size_t)mr * S::LDV + 4 * S::NB * S::CW + S::NB * S::CW + S::NB * S::NB + 4 * S::NB + 64 + N + 1;
  return d * sizeof(double) + sizeof(int) * (2 * N + 3 * S::NB + 1);
}

// Cross-lane steps of the panel's reductions by DPP on the vector ALU (a
// shuffle is a round trip through the LDS crossbar, and the column steps of
// a panel form one dependent chain).  A butterfly over xor 1, 2, 4 leaves
// equal values in every quad after its first two steps, so the third step
// may pair each lane with any lane of the other quad of its 8: the half-row
// mirror does, and gives the same sums as xor 4.  Likewise the row mirror
// stands in for xor 8 once each half-row holds one value.
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane l <-> 7 - l within 8
constexpr int DPP_MIRROR = 0x140;       // lane l <-> 15 - l within 16
template <int CTRL> __device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ double dpp_dbl(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_int<CTRL>((int)(b & 0xffffffffll)), hi = dpp_int<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sum over each group of 8 lanes, in every lane of the group, with the pairs
// and the order of a butterfly over xor 1, 2, 4; all 8 lanes must be active
__device__ __forceinline__ double sum8(double v) {
  v += dpp_dbl<DPP_XOR1>(v);
  v += dpp_dbl<DPP_XOR2>(v);
  v += dpp_dbl<DPP_HALF_MIRROR>(v);
  return v;
}

// Unblocked Householder on the LDS panel V[0..m) x [0..w): on return the
// strict lower part of the first weff columns holds v (v_j = 1 implicit),
// beta[j] = R_jj, tau[j]; the function returns weff.  Eight threads own each
// column.  With PIVOT the panel's columns are also pivoted (largest remaining
// norm first); the owners recompute their column's norm while applying each
// reflector, and the swaps are recorded in swp[j] for the rows above the
// panel.  The panel ends early (weff < w) at the first step whose best
// in-panel norm is below nuout, the largest norm outside the panel at its
// start: from there an outside column might be the larger.  Columns
// [weff, w) then hold the remaining rows updated by the weff reflectors, and
// pn[q] their squared norms over rows >= weff.
// Reflector j is formed on the fly (x_r times its scale) where it is used
// and stored once after the panel, so a column step needs one barrier (two
// with pivoting); the stored values are the same products.
template <class S, bool PIVOT>
__device__ __forceinline__ int panel_factor(const Lds &s, int m, int w, int *swp) {
  constexpr int LDV = S::LDV;
  const int t = threadIdx.x, sub = t & 7, qo = t >> 3;
  double *scl = s.red;   // [w] scale of each reflector column, applied after the panel
  // pn[q]: norm^2 of column q over rows >= j; pg[q]: over rows > j
  {
    const int q = qo;
    double a0 = 0.0, a1 = 0.0;
    if (q < w)
      for (int r = sub; r < m; r += 8) { const double x = s.V[r * LDV + q]; a0 += x * x; if (r > 0) a1 += x * x; }
    a0 = sum8(a0);
    a1 = sum8(a1);
    if (q < w && sub == 0) { s.pn[q] = a0; s.pg[q] = a1; }
    __syncthreads();
  }
  int weff = w;
  for (int j = 0; j < w; ++j) {
    // pivot: every wavefront finds the first column of largest norm among
    // j..w-1 (lane q holds column j + q; w <= 64; a NaN norm ranks last, so
    // the order is total and the result does not depend on the order of the
    // reduction).  The norms of columns > j are recomputed by their owners
    // below, so pn / pg are not permuted: the norm of the column moved to j is
    // read at its old position p.
    int p = j;
    if (PIVOT) {
      const int lane = t & 63;
      double best = (j + lane < w) ? rank_key(s.pn[j + lane]) : -1.0;
      p = j + lane;
      auto take = [&](double ob, int op) {
        if (ranks_before(ob, op, best, p)) { best = ob; p = op; }
      };
      take(dpp_dbl<DPP_XOR1>(best), dpp_int<DPP_XOR1>(p));
      take(dpp_dbl<DPP_XOR2>(best), dpp_int<DPP_XOR2>(p));
      take(dpp_dbl<DPP_HALF_MIRROR>(best), dpp_int<DPP_HALF_MIRROR>(p));
      take(dpp_dbl<DPP_MIRROR>(best), dpp_int<DPP_MIRROR>(p));
      take(__shfl_xor(best, 16, 64), __shfl_xor(p, 16, 64));
      take(__shfl_xor(best, 32, 64), __shfl_xor(p, 32, 64));
      // every lane of every wavefront holds the same best: the exit is uniform
      if (j > 0 && best < s.nuout[0]) { weff = j; break; }
      if (p != j) {
        for (int r = t; r < m; r += QT) {
          const double a = s.V[r * LDV + j];
          s.V[r * LDV + j] = s.V[r * LDV + p];
          s.V[r * LDV + p] = a;
        }
      }
      if (t == 0) swp[j] = p;
      __syncthreads();
    }
    const double xn2 = s.pg[p];
    const double x0 = s.V[j * LDV + j];
    double tj = 0.0, bj = x0, scale = 0.0;
    if (xn2 > 0.0) {
      bj = (x0 >= 0.0 ? -1.0 : 1.0) * sqrt(x0 * x0 + xn2);
      tj = (bj - x0) / bj;
      scale = 1.0 / (x0 - bj);
    }
    if (t == 0) { s.tau[j] = tj; s.beta[j] = bj; scl[j] = scale; }
    const int q = j + 1 + qo;
    double a1 = 0.0, head = 0.0;   // norms of column q over rows > j+1 and its row j+1
    if (q < w) {
      // eight, then four rows per iteration: their loads are issued
      // together, the sums keep the row order
      double acc = (sub == 0) ? s.V[j * LDV + q] : 0.0;
      int r = j + 1 + sub;
      for (; r + 56 < m; r += 64) {
        double x[8], c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { x[u] = s.V[(r + 8 * u) * LDV + j] * scale; c[u] = s.V[(r + 8 * u) * LDV + q]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u] * c[u];
      }
      for (; r + 24 < m; r += 32) {
        double x[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { x[u] = s.V[(r + 8 * u) * LDV + j] * scale; c[u] = s.V[(r + 8 * u) * LDV + q]; }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += x[u] * c[u];
      }
      for (; r < m; r += 8) acc += (s.V[r * LDV + j] * scale) * s.V[r * LDV + q];
      acc = sum8(acc);
      const double f = tj * acc;
      if (sub == 0) s.V[j * LDV + q] -= f;
      r = j + 1 + sub;
      for (; r + 56 < m; r += 64) {
        double x[8], c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { x[u] = s.V[(r + 8 * u) * LDV + j] * scale; c[u] = s.V[(r + 8 * u) * LDV + q]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double v = c[u] - f * x[u];
          s.V[(r + 8 * u) * LDV + q] = v;
          if (r + 8 * u > j + 1) a1 += v * v; else head = v;
        }
      }
      for (; r + 24 < m; r += 32) {
        double x[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { x[u] = s.V[(r + 8 * u) * LDV + j] * scale; c[u] = s.V[(r + 8 * u) * LDV + q]; }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double v = c[u] - f * x[u];
          s.V[(r + 8 * u) * LDV + q] = v;
          if (r + 8 * u > j + 1) a1 += v * v; else head = v;
        }
      }
      for (; r < m; r += 8) {
        const double v = s.V[r * LDV + q] - f * (s.V[r * LDV + j] * scale);
        s.V[r * LDV + q] = v;
        if (r > j + 1) a1 += v * v; else head = v;
      }
    }
    a1 = sum8(a1);
    head = sum8(head);
    if (q < w && sub == 0) { s.pg[q] = a1; s.pn[q] = a1 + head * head; }
    __syncthreads();
  }
  // store the reflectors: v_r = x_r * scale below the diagonal
  for (int e = t; e < m * w; e += QT) {
    const int r = e / w, jj = e % w;
    if (r > jj && jj < weff) s.V[r * LDV + jj] *= scl[jj];
  }
  __syncthreads();
  return weff;
}

// Write the panel to global (factored columns q < weff: R on and above the
// diagonal, v below; columns [weff, w): their updated values) and turn LDS V
// into the clean reflector block of the weff factored columns (1 on the
// diagonal, zeros above and in the padding up to mr x NB).
template <class S>
__device__ __forceinline__ void panel_store_clean(const Lds &s, double *A, int N, int c0, int m, int w, int weff,
                                                  int mr) {
  constexpr int LDV = S::LDV;
  for (int e = threadIdx.x; e < m * w; e += QT) {
    const int r = e / w, q = e % w;
    A[(long)(c0 + r) * N + c0 + q] = (r == q && q < weff) ? s.beta[q] : s.V[r * LDV + q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < mr * S::NB; e += QT) {
    const int r = e / S::NB, q = e % S::NB;
    const double v = (q >= weff || r >= m || r < q) ? 0.0 : (r == q ? 1.0 : s.V[r * LDV + q]);
    s.V[r * LDV + q] = v;
  }
  __syncthreads();
}

template <class S>
__device__ __forceinline__ void panel_load_clean(const Lds &s, const double *A, int N, int c0, int m, int w, int mr) {
  constexpr int LDV = S::LDV;
  // unconditional loads from clamped addresses, eight in flight per thread
#pragma unroll 8
  for (int e = threadIdx.x; e < mr * S::NB; e += QT) {
    const int r = e / S::NB, q = e % S::NB;
    const double a = A[(long)(c0 + min(r, m - 1)) * N + c0 + min(q, w - 1)];
    const double v = (q >= w || r >= m || r < q) ? 0.0 : (r == q ? 1.0 : a);
    s.V[r * LDV + q] = v;
  }
  __syncthreads();
}

// T (upper triangular) of Q_p = I - V T V^T:
// T_jj = tau_j,  T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j).
// The Gram matrix V^T V comes from FP64 MFMA (K split over the wavefronts).
template <class S>
__device__ __forceinline__ void build_T(const Lds &s, int m, int w, int mr) {
  constexpr int LDV = S::LDV, NB = S::NB, WT = S::WT;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, l16 = lane & 15, lq = lane >> 4;
  double *part = s.Wp;                    // [4][NB][NB] partial Gram matrices
  double *gram = s.Wp + 4 * NB * NB;      // [NB][NB]
  {
    const int kq = mr / 4, kb = wv * kq;
    M64::acc_t g[WT][WT];
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b) g[a][b] = M64::acc_t{0, 0, 0, 0};
    for (int k0 = kb; k0 < kb + kq; k0 += 4) {
      const int k = k0 + lq;
      double va[WT];
#pragma unroll
      for (int a = 0; a < WT; ++a) va[a] = s.V[k * LDV + 16 * a + l16];
#pragma unroll
      for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b) g[a][b] = M64::mac(va[a], va[b], g[a][b]);
    }
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[(wv * NB + 16 * a + M64::row(lane, r)) * NB + 16 * b + l16] = g[a][b][r];
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += QT) {
    gram[e] = (part[e] + part[NB * NB + e]) + (part[2 * NB * NB + e] + part[3 * NB * NB + e]);
    s.T[e] = 0.0;
  }
  __syncthreads();
  // the recurrence runs in wavefront 0, lane t holding row t of T in
  // registers (w <= NB <= 32).  Row t is zero left of the diagonal, so
  // summing from q = 0 adds exact zeros before the terms q >= t: the sums
  // are those of the recurrence taken from q = t.
  if (wv == 0) {
    double tr[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) tr[q] = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < w) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < j; ++q) v += tr[q] * gram[q * NB + j];
        const double tj = s.tau[j];
        tr[j] = t < j ? -tj * v : (t == j ? tj : 0.0);
      }
    }
    if (t < NB) {
#pragma unroll
      for (int q = 0; q < NB; ++q) s.T[t * NB + q] = tr[q];
    }
  }
  __syncthreads();
  (void)m;
}

// Apply (I - V op(T) V^T) to columns [c0, c1) of X (rows r0..r0+m), row
// stride ldx.  TRANS_T: op(T) = T^T (Q_p^T, used while factoring), else T
// (Q_p, used to form Q).  With NORMS, the squared norms of the updated
// columns over rows >= r0 + nskip are left in s.norms[col].
template <class S, bool TRANS_T, bool NORMS>
__device__ __forceinline__ void apply_block(const Lds &s, double *X, long ldx, int r0, int m, int mr, int c0, int c1, int nskip) {
  constexpr int LDV = S::LDV, NB = S::NB, CW = S::CW, CT = S::CT, WT = S::WT, RTW = S::RTW;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int rtiles = mr / 16;
  for (int cc = c0; cc < c1; cc += CW) {
    // 1. chunk into registers (accumulator layout): tile (rt, u), reg r holds
    //    row 16 rt + lq + 4 r, column cc + 16 u + l16
    M64::acc_t cr[RTW][CT];
#pragma unroll
    for (int a = 0; a < RTW; ++a) {
      const int rt = wv + 4 * a;
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const int col = cc + 16 * u + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + lq + 4 * r;
          cr[a][u][r] = (rt < rtiles && row < m && col < c1) ? X[(long)(r0 + row) * ldx + col] : 0.0;
        }
      }
    }
    // 2. this wave's partial W = V^T C over its row tiles
    M64::acc_t wacc[WT][CT];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int u = 0; u < CT; ++u) wacc[i][u] = M64::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < RTW; ++a) {
      const int rt = wv + 4 * a;
      if (rt < rtiles) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int k = 16 * rt + 4 * st + lq;
#pragma unroll
          for (int i = 0; i < WT; ++i) {
            const double av = s.V[k * LDV + 16 * i + l16];
#pragma unroll
            for (int u = 0; u < CT; ++u) wacc[i][u] = M64::mac(av, cr[a][u][st], wacc[i][u]);
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int u = 0; u < CT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) s.Wp[(wv * NB + 16 * i + M64::row(lane, r)) * CW + 16 * u + l16] = wacc[i][u][r];
    __syncthreads();
    // 3. W = sum of partials; W2 = -op(T) W
    for (int e = t; e < NB * CW; e += QT)
      s.Wp[e] = (s.Wp[e] + s.Wp[NB * CW + e]) + (s.Wp[2 * NB * CW + e] + s.Wp[3 * NB * CW + e]);
    __syncthreads();
    for (int e = t; e < NB * CW; e += QT) {
      const int i = e / CW, q = e % CW;
      double acc = 0.0;
      if (TRANS_T) {
        for (int k = 0; k <= i; ++k) acc += s.T[k * NB + i] * s.Wp[k * CW + q];
      } else {
        for (int k = i; k < NB; ++k) acc += s.T[i * NB + k] * s.Wp[k * CW + q];
      }
      s.W2[e] = -acc;
    }
    __syncthreads();
    // 4. C += V W2 in registers, store, optional norms
    double nrm[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) nrm[u] = 0.0;
#pragma unroll
    for (int a = 0; a < RTW; ++a) {
      const int rt = wv + 4 * a;
      if (rt < rtiles) {
#pragma unroll
        for (int k0 = 0; k0 < NB; k0 += 4) {
          const double av = s.V[(16 * rt + l16) * LDV + k0 + lq];
#pragma unroll
          for (int u = 0; u < CT; ++u) cr[a][u] = M64::mac(av, s.W2[(k0 + lq) * CW + 16 * u + l16], cr[a][u]);
        }
#pragma unroll
        for (int u = 0; u < CT; ++u) {
          const int col = cc + 16 * u + l16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * rt + lq + 4 * r;
            if (row < m && col < c1) {
              X[(long)(r0 + row) * ldx + col] = cr[a][u][r];
              if (NORMS && row >= nskip) nrm[u] += cr[a][u][r] * cr[a][u][r];
            }
          }
        }
      }
    }
    if (NORMS) {
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        double v = nrm[u];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lq == 0) s.npart[wv * CW + 16 * u + l16] = v;
      }
      __syncthreads();
      for (int q = t; q < CW; q += QT)
        if (cc + q < c1) s.norms[cc + q] = (s.npart[q] + s.npart[CW + q]) + (s.npart[2 * CW + q] + s.npart[3 * CW + q]);
    }
    __syncthreads();
  }
}

// The same product for N <= 16 MT, one 16-column tile per wavefront at a
// time.  The tile is held over all rows in accumulator layout (register r of
// lane (lq, l16): row 16 rt + lq + 4 r, column l16), which is also the layout
// of an MFMA B operand whose k-step st takes register st.  So W = V^T C,
// W2 = op(T) W and C -= V W2 all run on MFMA from the wavefront's own
// registers; only V and T are read from LDS, and no data passes between
// wavefronts.  With NORMS each column's squared norm over rows >= nskip is
// summed within the wavefront.
template <class S, bool TRANS_T, bool NORMS>
__device__ __forceinline__ void apply_cols(const Lds &s, double *X, long ldx, int r0, int m, int mr, int c0, int c1, int nskip) {
  constexpr int LDV = S::LDV, NB = S::NB, WT = S::WT, MT = S::MT;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int rtiles = mr / 16;
  for (int cc = c0 + 16 * wv; cc < c1; cc += 16 * (QT / 64)) {
    const int col = cc + l16;
    const bool cok = col < c1;
    // rows are walked with one running offset (the empty asm keeps the
    // compiler from materialising all 4 MT row addresses at once)
    const long step = 4 * ldx, off0 = (long)(r0 + lq) * ldx + col;
    M64::acc_t cr[MT];
    {
      long off = off0;
#pragma unroll
      for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + lq + 4 * r;
          cr[rt][r] = (rt < rtiles && row < m && cok) ? X[off] : 0.0;
          off += step;
          asm volatile("" : "+v"(off));
        }
    }
    // W = V^T C  (NB x 16)
    M64::acc_t w[WT];
#pragma unroll
    for (int i = 0; i < WT; ++i) w[i] = M64::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
      if (rt < rtiles) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int k = 16 * rt + 4 * st + lq;
#pragma unroll
          for (int i = 0; i < WT; ++i) w[i] = M64::mac(s.V[k * LDV + 16 * i + l16], cr[rt][st], w[i]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);   // keep one row tile's operands live at a time
    }
    // W2 = op(T) W  (T upper triangular, zero below the diagonal)
    M64::acc_t w2[WT];
#pragma unroll
    for (int i = 0; i < WT; ++i) w2[i] = M64::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int it = 0; it < WT; ++it)
#pragma unroll
      for (int kt = 0; kt < WT; ++kt)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int i = 16 * it + l16, k = 16 * kt + 4 * st + lq;
          w2[it] = M64::mac(TRANS_T ? s.T[k * NB + i] : s.T[i * NB + k], w[kt][st], w2[it]);
        }
    // C -= V W2
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) w2[i][r] = -w2[i][r];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
      if (rt < rtiles) {
#pragma unroll
        for (int kt = 0; kt < WT; ++kt)
#pragma unroll
          for (int st = 0; st < 4; ++st)
            cr[rt] = M64::mac(s.V[(16 * rt + l16) * LDV + 16 * kt + 4 * st + lq], w2[kt][st], cr[rt]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    double nrm = 0.0;
    {
      long off = off0;
#pragma unroll
      for (int rt = 0; rt < MT; ++rt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + lq + 4 * r;
          if (rt < rtiles && row < m && cok) {
            X[off] = cr[rt][r];
            if (NORMS && row >= nskip) nrm += cr[rt][r] * cr[rt][r];
          }
          off += step;
          asm volatile("" : "+v"(off));
        }
      }
    }
    if (NORMS) {
      nrm += __shfl_xor(nrm, 16, 64);
      nrm += __shfl_xor(nrm, 32, 64);
      if (lq == 0 && cok) s.norms[col] = nrm;
    }
  }
  __syncthreads();
}

template <class S, bool TRANS_T, bool NORMS>
__device__ __forceinline__ void apply(const Lds &s, double *X, long ldx, int r0, int m, int mr, int c0, int c1, int nskip) {
  if constexpr (S::COLS) apply_cols<S, TRANS_T, NORMS>(s, X, ldx, r0, m, mr, c0, c1, nskip);
  else apply_block<S, TRANS_T, NORMS>(s, X, ldx, r0, m, mr, c0, c1, nskip);
}

// Swap the NB remaining columns of largest current norm (ties: lower physical
// index first) into positions [c0, c0 + w), in order of decreasing norm; the
// columns they displace take the vacated positions (k-th displaced column,
// by position, to the k-th vacated position).  Whole columns move, so the R
// rows above the panel stay consistent.  The chosen columns are staged in
// LDS: rows >= c0 straight into the panel layout (V[r - c0], zero-padded to
// mr x NB), which is what the factorisation loads, and rows < c0 below them
// (V[m + r]) until they are written back to A.  The panel rows of A itself
// are written when the factored panel is stored.
template <class S>
__device__ __forceinline__ void select_panel(const Lds &s, double *A, int N, int c0, int w, int m, int mr) {
  constexpr int LDV = S::LDV;
  const int t = threadIdx.x;
  int *rank = s.sel;          // [N]
  int *src = s.sel + N;       // [NB]  chosen column of each rank
  int *mv_from = src + S::NB; // [NB]  displaced column positions
  int *mv_to = mv_from + S::NB;
  int *nmv = mv_to + S::NB;
  // a NaN norm ranks last, so that the comparison stays a strict total order
  // and the ranks of the remaining columns are a permutation of 0..N-c0-1
  // (the counting loops read LDS words that every lane shares; unrolled, a
  // group of reads is in flight at once instead of one read per step)
  if (t == 0) s.nuout[0] = 0.0;   // no column outside the panel
  for (int q = c0 + t; q < N; q += QT) {
    const double nq = rank_key(s.norms[q]);
    int r = 0;
#pragma unroll 16
    for (int p = c0; p < N; ++p) r += ranks_before(rank_key(s.norms[p]), p, nq, q);
    rank[q] = r;
  }
  __syncthreads();
  for (int q = c0 + t; q < N; q += QT) {
    const int r = rank[q];
    if (r < w) src[r] = q;
    if (r == w) s.nuout[0] = isnan(s.norms[q]) ? 0.0 : s.norms[q];   // largest norm left outside
    if (r < w && q >= c0 + w) {          // vacated position: k-th among them
      int k = 0;
#pragma unroll 16
      for (int p = c0 + w; p < q; ++p) k += rank[p] < w;
      mv_to[k] = q;
    }
    if (r >= w && q < c0 + w) {          // displaced column: k-th among them
      int k = 0;
#pragma unroll 16
      for (int p = c0; p < q; ++p) k += rank[p] >= w;
      mv_from[k] = q;
    }
  }
  if (t == 0) {
    int k = 0;
#pragma unroll 16
    for (int p = c0; p < c0 + w; ++p) k += rank[p] >= w;
    *nmv = k;
  }
  __syncthreads();
  const int nd = min(*nmv, w);
  // stage chosen columns (all rows), move the displaced ones, write back
  // the rows above the panel.  The columns are strided in the row-major
  // matrix, so each element is its own memory access: all of a thread's loads
  // (at most GM) are issued before the first store, and each pass costs one
  // global round trip instead of one per group of loads.
  constexpr int GM = 32;
  static_assert(S::MT * 16 * S::NB <= GM * QT, "a thread's share of a panel exceeds the gather registers");
  {
    double g[GM];
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT;
      if (e < N * w) {
        const int r = e / w, i = e % w;
        g[u] = A[(long)r * N + src[i]];
      }
    }
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT;
      if (e < N * w) {
        const int r = e / w, i = e % w;
        s.V[(r >= c0 ? r - c0 : m + r) * LDV + i] = g[u];
      }
    }
  }
  int o_i = 0, o_d = 0;
  double n_i = 0.0, n_d = 0.0;
  if (t < w) { o_i = s.orig[src[t]]; n_i = s.norms[src[t]]; }
  if (t < nd) { o_d = s.orig[mv_from[t]]; n_d = s.norms[mv_from[t]]; }
  __syncthreads();
  {
    double g[GM];
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT;
      if (e < N * nd) {
        const int r = e / nd, i = e % nd;
        g[u] = A[(long)r * N + mv_from[i]];
      }
    }
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT;
      if (e < N * nd) {
        const int r = e / nd, i = e % nd;
        A[(long)r * N + mv_to[i]] = g[u];
      }
    }
  }
  if (t < nd) { s.orig[mv_to[t]] = o_d; s.norms[mv_to[t]] = n_d; }
  __syncthreads();
  for (int e = t; e < c0 * w; e += QT) {
    const int r = e / w, i = e % w;
    A[(long)r * N + c0 + i] = s.V[(m + r) * LDV + i];
  }
  if (t < w) { s.orig[c0 + t] = o_i; s.norms[c0 + t] = n_i; }
  __syncthreads();
  // zero padding of the panel: rows [m, mr) (which held the rows above the
  // panel) and columns [w, NB)
  for (int e = t; e < mr * S::NB; e += QT) {
    const int r = e / S::NB, q = e % S::NB;
    if (r >= m || q >= w) s.V[r * LDV + q] = 0.0;
  }
  __syncthreads();
}

// factor A (N x N, in place) panel by panel.  Panel k's T (w_k x w_k,
// packed) is saved to Tsave at the sum of the earlier w_j^2, and with PIVOT
// its start and width to plist[2k], plist[2k + 1] (panels have variable
// width there).
// Returns the number of panels.
template <class S, bool PIVOT>
__device__ __forceinline__ int factor(const Lds &s, double *A, double *Tsave, int *plist, int N) {
  constexpr int NB = S::NB, LDV = S::LDV;
  int c0 = 0, np = 0;
  long toff = 0;
  while (c0 < N) {
    const int w = min(NB, N - c0), m = N - c0, mr = round16(m);
    if (PIVOT) {
      select_panel<S>(s, A, N, c0, w, m, mr);   // leaves the panel in V
    } else {
#pragma unroll 8
      for (int e = threadIdx.x; e < mr * NB; e += QT) {
        const int r = e / NB, q = e % NB;
        const double a = A[(long)(c0 + min(r, m - 1)) * N + c0 + min(q, w - 1)];
        s.V[r * LDV + q] = (r < m && q < w) ? a : 0.0;
      }
      __syncthreads();
    }
    const int weff = panel_factor<S, PIVOT>(s, m, w, s.sel);
    if (PIVOT) {
      // the in-panel swaps also permute the R rows above the panel and orig[]:
      // as one gather per row, column q of the result from column idx[q]
      int *idx = s.sel + NB;
      if (threadIdx.x == 0) {
        for (int q = 0; q < w; ++q) idx[q] = q;
        for (int j = 0; j < weff; ++j) {
          const int p = s.sel[j];
          if (p != j) {
            const int a = idx[j]; idx[j] = idx[p]; idx[p] = a;
            const int o = s.orig[c0 + j]; s.orig[c0 + j] = s.orig[c0 + p]; s.orig[c0 + p] = o;
          }
        }
        plist[2 * np] = c0;
        plist[2 * np + 1] = weff;
      }
      __syncthreads();
      for (int r = threadIdx.x; r < c0; r += QT) {
        double v[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < w) v[q] = A[(long)r * N + c0 + idx[q]];
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < w) A[(long)r * N + c0 + q] = v[q];
      }
      // the panel's unfactored columns rejoin the trailing matrix with their
      // norms over rows >= c0 + weff
      for (int q = weff + threadIdx.x; q < w; q += QT) s.norms[c0 + q] = s.pn[q];
      __syncthreads();
    }
    panel_store_clean<S>(s, A, N, c0, m, w, weff, mr);
    build_T<S>(s, m, weff, mr);
    for (int e = threadIdx.x; e < weff * weff; e += QT) Tsave[toff + e] = s.T[(e / weff) * NB + e % weff];
    if (c0 + w < N) apply<S, true, PIVOT>(s, A, N, c0, m, mr, c0 + w, N, weff);
    toff += (long)weff * weff;
    c0 += weff;
    ++np;
  }
  return np;
}

template <class S>
__global__ __launch_bounds__(QT) void k_qr_udv(double *Xall, double *Tall, long tstride, double *Sall,
                                               double *Uall, double *Dall, double *RPall, int N) {
  extern __shared__ double smem[];
  const Lds s = carve<S>((char *)smem, N);
  const long NN = (long)N * N, b = blockIdx.x;
  double *X = Xall + b * NN, *U = Uall + b * NN, *RP = RPall + b * NN, *D = Dall + b * N;
  double *Ts = Tall + b * tstride;
  int *plist = (int *)(Sall + b * (long)N);   // qr_scratch_doubles(N) per matrix
  const int t = threadIdx.x;
  {
    for (int q = t; q < N; q += QT) {
      // sixteen rows' loads in flight per step; the sum keeps the row order
      double acc = 0.0;
      int r = 0;
      for (; r + 16 <= N; r += 16) {
        double x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = X[(long)(r + u) * N + q];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += x[u] * x[u];
      }
      for (; r < N; ++r) { const double x = X[(long)r * N + q]; acc += x * x; }
      s.norms[q] = acc;
      s.orig[q] = q;
    }
    __syncthreads();   // the panel selection reads every column's norm
  }
  const int np = factor<S, true>(s, X, Ts, plist, N);
  // D = diag R,  RP[i][orig[q]] = R[i][q] / R[i][i]
  for (int i = t; i < N; i += QT) D[i] = X[(long)i * N + i];
  // eight elements' loads in flight per step
  for (long e0 = t; e0 < NN; e0 += 8L * QT) {
    double xv[8], dv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const long e = e0 + (long)k * QT;
      xv[k] = dv[k] = 1.0;
      if (e < NN) {
        const int i = (int)(e / N);
        xv[k] = X[e];
        dv[k] = X[(long)i * N + i];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const long e = e0 + (long)k * QT;
      if (e < NN) {
        const int i = (int)(e / N), q = (int)(e % N);
        const double v = q < i ? 0.0 : (q == i ? 1.0 : xv[k] / dv[k]);
        RP[(long)i * N + s.orig[q]] = v;
      }
    }
  }
  // Q = Q_0 Q_1 ... applied in reverse order to the identity
  for (long e = t; e < NN; e += QT) U[e] = ((e / N) == (e % N)) ? 1.0 : 0.0;
  __syncthreads();
  long toff = 0;
  for (int p = 0; p < np; ++p) toff += (long)plist[2 * p + 1] * plist[2 * p + 1];
  for (int p = np - 1; p >= 0; --p) {
    const int c0 = plist[2 * p], w = plist[2 * p + 1], m = N - c0, mr = round16(m);
    toff -= (long)w * w;
    panel_load_clean<S>(s, X, N, c0, m, w, mr);
    for (int e = t; e < S::NB * S::NB; e += QT) {
      const int i = e / S::NB, q = e % S::NB;
      s.T[e] = (i < w && q < w) ? Ts[toff + i * w + q] : 0.0;
    }
    __syncthreads();
    apply<S, false, false>(s, U, N, c0, m, mr, c0, N, 0);
  }
}

// Back substitution U Z = Y in place of Y (B), U upper triangular in M with
// row i of U in row rowmap[i] of M, block rows of NB from the bottom: the
// block row of U right of the diagonal block is staged in LDS for the MFMA
// update, the diagonal block solved per column.
template <class S>
__device__ __forceinline__ void back_substitute(const Lds &s, const double *M, double *B, int N, const int *rowmap) {
  constexpr int NB = S::NB;
  auto mrow = [&](int i) { return rowmap[i]; };
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int np = (N + NB - 1) / NB;
  double *Rd = s.T;   // diagonal block of U, [NB][NB]
  // the panel and partial-sum areas (contiguous, free after the factorisation)
  // hold the block row of U right of the diagonal block; the row stride is
  // 2 mod 32 doubles so that the MFMA operand reads hit distinct banks
  double *Rs = s.V;
  const int RLD = ((N + 31) / 32) * 32 + 2;
  for (int p = np - 1; p >= 0; --p) {
    const int r0 = p * NB, w = min(NB, N - r0), k0 = r0 + w, kn = N - k0;
    if (kn > 0) {   // Y_p -= U[r0:r0+w, k0:N] Z[k0:N, :]
#pragma unroll 8
      for (int e = t; e < NB * kn; e += QT) {
        const int i = e / kn, k = e % kn;
        const double a = M[(long)mrow(r0 + min(i, w - 1)) * N + k0 + k];
        Rs[i * RLD + k] = (i < w) ? a : 0.0;
      }
      __syncthreads();
      // one 16-column tile per wavefront at a time, for every row tile of the
      // block row: each element of Z is loaded once, four k-steps ahead
      const int ctiles = (N + 15) / 16;
      for (int tc = wv; tc < ctiles; tc += QT / 64) {
        const int cj = tc * 16 + l16;
        M64::acc_t acc[S::WT];
#pragma unroll
        for (int tr = 0; tr < S::WT; ++tr) acc[tr] = M64::acc_t{0, 0, 0, 0};
        int kk = 0;
        for (; kk + 16 <= kn; kk += 16) {
          double bz[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) bz[u] = (cj < N) ? B[(long)(k0 + kk + 4 * u + lq) * N + cj] : 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int tr = 0; tr < S::WT; ++tr)
              acc[tr] = M64::mac(Rs[(tr * 16 + l16) * RLD + kk + 4 * u + lq], bz[u], acc[tr]);
        }
        for (; kk < kn; kk += 4) {
          const int k = kk + lq;
          const double bb = (k < kn && cj < N) ? B[(long)(k0 + k) * N + cj] : 0.0;
#pragma unroll
          for (int tr = 0; tr < S::WT; ++tr)
            acc[tr] = M64::mac(k < kn ? Rs[(tr * 16 + l16) * RLD + k] : 0.0, bb, acc[tr]);
        }
#pragma unroll
        for (int tr = 0; tr < S::WT; ++tr)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + tr * 16 + M64::row(lane, r);
            if (row < r0 + w && cj < N) B[(long)row * N + cj] -= acc[tr][r];
          }
      }
    }
    for (int e = t; e < NB * NB; e += QT) {
      const int i = e / NB, q = e % NB;
      Rd[e] = (i < w && q < w) ? M[(long)mrow(r0 + i) * N + r0 + q] : 0.0;
    }
    __syncthreads();
    for (int q = t; q < N; q += QT) {   // one right-hand side column per thread
      double z[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) z[i] = (i < w) ? B[(long)(r0 + i) * N + q] : 0.0;
#pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        if (i < w) {
          double acc = z[i];
#pragma unroll
          for (int k = i + 1; k < NB; ++k) acc -= Rd[i * NB + k] * z[k];
          z[i] = acc / Rd[i * NB + i];
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < w) B[(long)(r0 + i) * N + q] = z[i];
    }
    __syncthreads();
  }
}

// Solve M Z = B by LU with partial pivoting: Z in B, M overwritten by its
// factors; one workgroup per matrix.  Right-looking, in panels of NB columns.
// Rows are never moved: perm[i] (LDS) is the row of M and B that holds
// logical row i.  A panel is factored in LDS in the order its rows were
// loaded, each pivot chosen among the rows not yet chosen (largest |a|, a NaN
// last, ties to the lower position: the order of qr_order.h), and stored back
// to the rows it came from.  B's columns go along as further columns of the
// trailing matrix, so after the last panel B holds L^-1 P B; its rows are
// then put in logical order and U Z = L^-1 P B is solved by back_substitute
// with U's rows read through perm.
template <class S>
__global__ __launch_bounds__(QT) void k_lu_solve(double *Mall, double *Ball, int N) {
  constexpr int NB = S::NB, LDV = S::LDV;
  constexpr int RPT = S::MT * 16 / QT;   // panel rows per thread (1 or 2)
  static_assert(RPT * QT == S::MT * 16, "panel rows not divisible over the threads");
  extern __shared__ double smem[];
  const Lds s = carve<S>((char *)smem, N);
  const long NN = (long)N * N, b = blockIdx.x;
  double *M = Mall + b * NN, *B = Ball + b * NN;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  int *perm = s.orig;        // [N] logical row -> stored row
  int *lrow = s.sel;         // [NB] panel position of the j-th pivot
  int *loc = s.sel + NB;     // [N] panel position of the i-th row left after the panel
  int *redi = loc + N;       // [4] pivot candidates by wavefront
  int *cnt = redi + 4;       // [4] rows left per wavefront
  double *redv = s.red;      // [4]
  double *L11 = s.T;         // [NB][NB] the panel's unit lower block, logical order
  for (int i = t; i < N; i += QT) perm[i] = i;
  __syncthreads();
  // a thread's share of an N x NB block (panel loads, the reordering of B):
  // all of its loads are issued before the first store
  constexpr int GM = S::MT * 16 * NB / QT;
  double g[GM];
  for (int c0 = 0; c0 < N; c0 += NB) {
    const int w = min(NB, N - c0), m = N - c0, mt = m - w;
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT, r = e / NB, q = e % NB;
      g[u] = (r < m && q < w) ? M[(long)perm[c0 + r] * N + c0 + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT, r = e / NB, q = e % NB;
      if (r < m) s.V[r * LDV + q] = g[u];
    }
    __syncthreads();
    // unblocked LU of the panel: a thread holds its rows in registers (the
    // column steps unrolled, so that every index is static); per step the
    // candidates meet through LDS, the chosen row is published there, and
    // the other rows take their multipliers and updates from it
    double rv[RPT][NB];
    bool chosen[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      chosen[k] = false;
      const int r = t + k * QT;
#pragma unroll
      for (int q = 0; q < NB; ++q) rv[k][q] = r < m ? s.V[r * LDV + q] : 0.0;
    }
    double *prow = s.Wp;   // [NB] the pivot row of the current step
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < w) {
        double best = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = t + k * QT;
          if (r < m && !chosen[k]) {
            const double key = rank_key(fabs(rv[k][j]));
            if (ranks_before(key, r, best, bi)) { best = key; bi = r; }
          }
        }
        auto take = [&](double ob, int op) {
          if (ranks_before(ob, op, best, bi)) { best = ob; bi = op; }
        };
        take(dpp_dbl<DPP_XOR1>(best), dpp_int<DPP_XOR1>(bi));
        take(dpp_dbl<DPP_XOR2>(best), dpp_int<DPP_XOR2>(bi));
        take(dpp_dbl<DPP_HALF_MIRROR>(best), dpp_int<DPP_HALF_MIRROR>(bi));
        take(dpp_dbl<DPP_MIRROR>(best), dpp_int<DPP_MIRROR>(bi));
        take(__shfl_xor(best, 16, 64), __shfl_xor(bi, 16, 64));
        take(__shfl_xor(best, 32, 64), __shfl_xor(bi, 32, 64));
        if (lane == 0) { redv[wv] = best; redi[wv] = bi; }
        __syncthreads();
        double pb = redv[0];
        int P = redi[0];
#pragma unroll
        for (int q = 1; q < 4; ++q)
          if (ranks_before(redv[q], redi[q], pb, P)) { pb = redv[q]; P = redi[q]; }
        if (t == 0) lrow[j] = P;
#pragma unroll
        for (int k = 0; k < RPT; ++k)
          if (t + k * QT == P) {
            chosen[k] = true;
#pragma unroll
            for (int q = j; q < NB; ++q) prow[q] = rv[k][q];
          }
        __syncthreads();
        const double piv = prow[j];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = t + k * QT;
          if (r < m && !chosen[k]) {
            const double l = rv[k][j] / piv;
            rv[k][j] = l;
#pragma unroll
            for (int q = j + 1; q < NB; ++q) rv[k][q] -= l * prow[q];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = t + k * QT;
      if (r < m) {
#pragma unroll
        for (int q = 0; q < NB; ++q) s.V[r * LDV + q] = rv[k][q];
      }
    }
    __syncthreads();
    // the rows left, in panel order, follow the pivots
    int before = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = t + k * QT;
      const bool left = r < m && !chosen[k];
      const unsigned long long bal = __ballot(left);
      if (lane == 0) cnt[wv] = __popcll(bal);
      __syncthreads();
      int off = before;
      for (int q = 0; q < wv; ++q) off += cnt[q];
      if (left) loc[off + __popcll(bal & ((1ull << lane) - 1ull))] = r;
      for (int q = 0; q < 4; ++q) before += cnt[q];
      __syncthreads();
    }
    // store the factored panel to its rows, the unit lower block in logical
    // order, then the new logical order of the rows c0..N-1
    for (int e = t; e < m * w; e += QT) {
      const int r = e / w, q = e % w;
      M[(long)perm[c0 + r] * N + c0 + q] = s.V[r * LDV + q];
    }
    for (int e = t; e < NB * NB; e += QT) {
      const int i = e / NB, q = e % NB;
      L11[e] = (i < w && q < i) ? s.V[lrow[i] * LDV + q] : 0.0;
    }
    int np[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = t + k * QT;
      np[k] = i < m ? perm[c0 + (i < w ? lrow[i] : loc[i - w])] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = t + k * QT;
      if (i < m) perm[c0 + i] = np[k];
    }
    __syncthreads();
    // L11^-1 (unit lower) into LDS, one column per thread of the first
    // wavefront by forward substitution (L11 is zero beyond w x w, so the
    // inverse is the identity there)
    double *Li = s.W2;   // [NB][NB]
    if (t < NB) {
      double y[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        double acc = i == t ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= L11[i * NB + k] * y[k];
        y[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) Li[i * NB + t] = y[i];
    }
    __syncthreads();
    // U12 = L11^-1 A12 for M's columns right of the panel and B's columns, on
    // FP64 MFMA: a wavefront holds a 16-column tile of A12 and overwrites it
    const int ncm = N - c0 - w;
    {
      const int tiles_m = (ncm + 15) / 16, tiles = tiles_m + (N + 15) / 16;
      for (int tc = wv; tc < tiles; tc += QT / 64) {
        double *A = tc < tiles_m ? M : B;
        const int cl = (tc < tiles_m ? tc : tc - tiles_m) * 16 + l16;
        const bool cin = cl < (tc < tiles_m ? ncm : N);
        const int col = tc < tiles_m ? c0 + w + cl : cl;
        double bz[NB / 4];
#pragma unroll
        for (int u = 0; u < NB / 4; ++u) {
          const int k = 4 * u + lq;
          bz[u] = (cin && k < w) ? A[(long)perm[c0 + k] * N + col] : 0.0;
        }
        M64::acc_t cv[NB / 16];
#pragma unroll
        for (int q = 0; q < NB / 16; ++q) {
          cv[q] = M64::acc_t{0, 0, 0, 0};
#pragma unroll
          for (int u = 0; u < NB / 4; ++u) cv[q] = M64::mac(Li[(q * 16 + l16) * NB + 4 * u + lq], bz[u], cv[q]);
        }
#pragma unroll
        for (int q = 0; q < NB / 16; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = q * 16 + M64::row(lane, r);
            if (row < w && cin) A[(long)perm[c0 + row] * N + col] = cv[q][r];
          }
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12 on FP64 MFMA: 16-column tiles per
    // wavefront; a tile's rows are loaded together, RC row tiles at a time,
    // and the products (-L21 from the panel in LDS, U12 held in registers)
    // accumulate into them
    if (mt > 0) {
      constexpr int RC = S::MT < 16 ? S::MT : 16;
      const int tiles_m = (ncm + 15) / 16, tiles = tiles_m + (N + 15) / 16;
      const int rtiles = (mt + 15) / 16;
      for (int tc = wv; tc < tiles; tc += QT / 64) {
        double *A = tc < tiles_m ? M : B;
        const int cl = (tc < tiles_m ? tc : tc - tiles_m) * 16 + l16;
        const bool cin = cl < (tc < tiles_m ? ncm : N);
        const int col = tc < tiles_m ? c0 + w + cl : cl;
        double bz[NB / 4];
#pragma unroll
        for (int u = 0; u < NB / 4; ++u) {
          const int k = 4 * u + lq;
          bz[u] = (cin && k < w) ? A[(long)perm[c0 + k] * N + col] : 0.0;
        }
        for (int t0 = 0; t0 < rtiles; t0 += RC) {
          M64::acc_t cv[RC];
#pragma unroll
          for (int q = 0; q < RC; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = (t0 + q) * 16 + M64::row(lane, r);
              cv[q][r] = (row < mt && cin) ? A[(long)perm[c0 + w + row] * N + col] : 0.0;
            }
#pragma unroll
          for (int q = 0; q < RC; ++q) {
            if (t0 + q < rtiles) {
              const int arow = (t0 + q) * 16 + l16;
              const int ar = arow < mt ? loc[arow] : 0;
#pragma unroll
              for (int u = 0; u < NB / 4; ++u) {
                const int k = 4 * u + lq;
                const double a = (arow < mt && k < w) ? -s.V[ar * LDV + k] : 0.0;
                cv[q] = M64::mac(a, bz[u], cv[q]);
              }
            }
          }
#pragma unroll
          for (int q = 0; q < RC; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = (t0 + q) * 16 + M64::row(lane, r);
              if (row < mt && cin) A[(long)perm[c0 + w + row] * N + col] = cv[q][r];
            }
        }
      }
    }
    __syncthreads();
  }
  // B's rows into logical order, NB columns at a time through LDS
  for (int cb = 0; cb < N; cb += NB) {
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT, i = e / NB, c = e % NB;
      g[u] = (i < N && cb + c < N) ? B[(long)perm[i] * N + cb + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT;
      if (e < N * NB) s.V[e] = g[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GM; ++u) {
      const int e = t + u * QT, i = e / NB, c = e % NB;
      g[u] = e < N * NB ? s.V[e] : 0.0;
      if (i < N && cb + c < N) B[(long)i * N + cb + c] = g[u];
    }
    __syncthreads();
  }
  back_substitute<S>(s, M, B, N, perm);
}

constexpr int SMALL_MAX_N = 256;
}  // namespace

size_t qr_tsave_doubles(int N) {
  const int nb = N <= SMALL_MAX_N ? ShapeS::NB : ShapeL::NB;
  return (size_t)((N + nb - 1) / nb) * nb * nb;
}

// the panel list of the pivoted factorisation: up to N panels of two ints
size_t qr_scratch_doubles(int N) { return (size_t)N; }

hipError_t qr_udv_blocked(double *X, double *Scr, double *Tsave, double *U, double *D, double *RP, int mats, int N,
                          hipStream_t s) {
  if (N > 512) return hipErrorInvalidValue;
  if ((N <= SMALL_MAX_N ? lds_bytes<ShapeS>(N) : lds_bytes<ShapeL>(N)) > 160 * 1024) return hipErrorInvalidValue;
  const long ts = (long)qr_tsave_doubles(N);
  if (N <= SMALL_MAX_N)
    hipLaunchKernelGGL(k_qr_udv<ShapeS>, dim3(mats), dim3(QT), lds_bytes<ShapeS>(N), s, X, Tsave, ts, Scr, U, D, RP,
                       N);
  else
    hipLaunchKernelGGL(k_qr_udv<ShapeL>, dim3(mats), dim3(QT), lds_bytes<ShapeL>(N), s, X, Tsave, ts, Scr, U, D, RP,
                       N);
  return hipGetLastError();
}

hipError_t lu_solve_blocked(double *M, double *B, int mats, int N, hipStream_t s) {
  if (N > 512) return hipErrorInvalidValue;
  if ((N <= SMALL_MAX_N ? lds_bytes<ShapeS>(N) : lds_bytes<ShapeL>(N)) > 160 * 1024) return hipErrorInvalidValue;
  if (N <= SMALL_MAX_N)
    hipLaunchKernelGGL(k_lu_solve<ShapeS>, dim3(mats), dim3(QT), lds_bytes<ShapeS>(N), s, M, B, N);
  else
    hipLaunchKernelGGL(k_lu_solve<ShapeL>, dim3(mats), dim3(QT), lds_bytes<ShapeL>(N), s, M, B, N);
  return hipGetLastError();
}


}  // namespace bss
