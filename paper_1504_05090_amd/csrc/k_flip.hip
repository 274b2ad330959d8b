// Flip phase of one time slice: Metropolis decisions on the Ising field with
// Sherman-Morrison updates of G delayed to rank k.
//
// One workgroup runs one Markov chain (both spins); thread j owns site j of
// the slice.  Per proposal the determinant ratio is
//   R = R_up R_dn,  R_sigma = 1 + (1 - G_sigma,jj) Delta_sigma,
//   Delta_sigma = e^{-2 sigma lambda h_j} - 1,
// and the flip is accepted iff u_j < R (u_j from Philox at counter
// (sweep, (l-1) N + j, 0, 0)).  With the updates delayed,
//   G = G0 - sum_m x_m y_m^T,
// and thread j keeps its rows of X and Y and its current diagonal element
// d_j = G_jj in registers.  Because every site's ratio depends only on its
// own d_j, all sites are tested in parallel and a wavefront ballot picks the
// first accepted site after the last one: the proposals rejected before it
// are exactly those the sequential visit would reject.  On acceptance at
// site i the new pair is
//   c = G0 e_i - X (Y^T e_i),  r = e_i^T G0 - (e_i^T X) Y^T,
//   x = (Delta/R)(e_i - c),    y = r,
// and every d_j drops by x_j y_j.  When k pairs are stored (and at the end of
// the slice) they are flushed into G0 by a rank-k MFMA product.
//
// Precision: the arithmetic (T) is FP64.  G is stored (S) in FP64, or in FP32
// for the FP32 slices of mixed precision: then G is converted on load and
// rounded to FP32 when the flush stores it, so the stored values carry one
// FP32 rounding relative to themselves.  With FP32 arithmetic the rank-k
// product would sum terms |x_m| |y_m| up to |Delta/R| max|G|^2 (~1e6 at
// 16 x 16, beta = 20, where max|G| reaches ~100) into entries of order 1,
// and its absolute rounding error of ~1e-1 turns determinant ratios negative.
#include <utility>

#include "common.h"
#include "kernels.h"

namespace bss {

namespace {

// G0 <- G0 - X Y^T for one spin, on 16x16x4 MFMA tiles with the G0 tile as
// the accumulator input (D = (-X) Y^T + G0).  Rows of -X are staged in LDS
// by their owners in blocks of fb rows, Y^T once; each wavefront loads a
// batch of G0 tiles before its MFMAs so that the global latencies overlap.
template <typename T, typename S, int KM>
__device__ void flush_spin(S *G, int N, int fb, const T (&xs)[KM], const T (&ys)[KM], T *Xs, T *Ys) {
  constexpr int TB = 8;   // tiles in flight per wavefront
  const int j = threadIdx.x, lane = j & 63, w = j >> 6, nw = blockDim.x >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int ldy = blockDim.x + 1;
  const bool own = j < N;
#pragma unroll
  for (int s = 0; s < KM; ++s) Ys[s * ldy + j] = own ? ys[s] : (T)0;
  typedef typename Mfma<T>::acc_t acc_t;
  const int ctiles = (N + 15) >> 4;
  for (int i0 = 0; i0 < N; i0 += fb) {
    __syncthreads();
    if (j >= i0 && j < i0 + fb) {
#pragma unroll
      for (int s = 0; s < KM; ++s) Xs[(j - i0) * (KM + 1) + s] = own ? -xs[s] : (T)0;
    }
    __syncthreads();
    const int nrb = min(fb, N - i0);
    const int ntiles = ((nrb + 15) >> 4) * ctiles;
    for (int base = w; base < ntiles; base += nw * TB) {
      acc_t acc[TB];
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int tile = base + nw * b;
        const int tr = tile / ctiles, tc = tile % ctiles;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + tr * 16 + Mfma<T>::row(lane, r), col = tc * 16 + l16;
          acc[b][r] = (tile < ntiles && row < i0 + nrb && col < N) ? (T)G[(long)row * N + col] : (T)0;
        }
      }
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int tile = base + nw * b;
        if (tile < ntiles) {
          const int tr = tile / ctiles, tc = tile % ctiles;
#pragma unroll
          for (int s0 = 0; s0 < KM; s0 += 4) {
            const int s = s0 + lq;
            T a = (T)0, bb = (T)0;
            if (s < KM) {
              a = Xs[(tr * 16 + l16) * (KM + 1) + s];
              bb = Ys[s * ldy + tc * 16 + l16];
            }
            acc[b] = Mfma<T>::mac(a, bb, acc[b]);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = i0 + tr * 16 + Mfma<T>::row(lane, r), col = tc * 16 + l16;
            if (row < i0 + nrb && col < N) G[(long)row * N + col] = (S)acc[b][r];
          }
        }
      }
    }
  }
  __syncthreads();
}

template <typename T, typename S, int KM, int MAXT>
__global__ __launch_bounds__(MAXT) void k_flip(FlipArgs a) {
  extern __shared__ char smem_raw[];
  T *Xs = (T *)smem_raw;                                  // [fb][KM+1]
  T *Ys = Xs + a.fb * (KM + 1);                           // [KM][blockDim+1]
  // per-acceptance exchange, double-buffered by the parity of the acceptance
  // so that one barrier separates consecutive acceptances
  __shared__ int first[2][16];
  __shared__ T bX[2][2][KM], bY[2][2][KM];
  __shared__ double bF[2][2];
  __shared__ double s_R[MAXT];     // accepted ratios, logged after the loop
  __shared__ double red[16];
  __shared__ int s_acc;

  const int N = a.N, j = threadIdx.x, lane = j & 63, w = j >> 6, nw = blockDim.x >> 6;
  const int c = blockIdx.x;
  const bool own = j < N;
  const long NN = (long)N * N;
  S *G[2] = {(S *)a.G + (2L * c) * NN, (S *)a.G + (2L * c + 1) * NN};
  int8_t *hl = a.h + ((long)c * a.Lam + (a.l - 1)) * N;
  const int64_t sweep = *a.sweep;

  int hj = own ? hl[j] : 1;
  double uj = 2.0;
  bool forced = false;
  long trace_idx = -1;
  if (own && a.trace_mode != 0) {
    const int64_t rel = sweep - *a.trace_base;
    if (rel >= 0 && rel < a.trace_sweeps)
      trace_idx = ((rel * a.chains_total + a.chain0 + c) * (long)a.Lam + (a.l - 1)) * N + j;
  }
  if (own) {
    if (a.trace_mode == 2) {
      if (trace_idx >= 0) forced = a.trace[trace_idx] != 0;
      else atomicOr(a.err, 8);     // replay past the supplied history
    } else {
      uj = uniform53(philox_word0((uint64_t)sweep, (uint64_t)(a.l - 1) * N + j, 0, 0, a.seed + (uint64_t)(a.chain0 + c), a.inst));
    }
  }
  T xs[2][KM], ys[2][KM];
#pragma unroll
  for (int s = 0; s < KM; ++s) { xs[0][s] = xs[1][s] = ys[0][s] = ys[1][s] = (T)0; }
  double d[2];
  d[0] = own ? (double)G[0][(long)j * N + j] : 0.0;
  d[1] = own ? (double)G[1][(long)j * N + j] : 0.0;
  bool mine = false;   // my site was accepted
  if (j == 0) s_acc = 0;
  __syncthreads();

  int m = 0, pos = 0, par = 0;
  int badj = 0;   // 1: ratio <= 0, 2: ratio not finite
  int softj = 0;  // 1: ratio <= 0 in a guarded FP32 slice (rejected, counted)
  for (;;) {
    bool acc = false;
    if (own && j >= pos) {
      const double du = hj > 0 ? a.dlt_up_p : a.dlt_up_m;
      const double dd = hj > 0 ? a.dlt_dn_p : a.dlt_dn_m;
      const double R = (1.0 + (1.0 - d[0]) * du) * (1.0 + (1.0 - d[1]) * dd);
      acc = (a.trace_mode == 2) ? forced : (uj < R);
      // the last evaluation is the site's proposal: every weight of eq. (3)
      // is positive at half filling, so a ratio that is not a finite positive
      // number is an error whether or not it is accepted
      softj = (a.fp32_guard && isfinite(R) && !(R > 0.0)) ? 1 : 0;
      badj = softj ? 0 : (!isfinite(R) ? 2 : (R > 0.0 ? 0 : 1));
    }
    const unsigned long long bal = __ballot(acc);
    if (lane == 0) first[par][w] = bal ? (w * 64 + __ffsll((long long)bal) - 1) : 0x7fffffff;
    __syncthreads();
    int ist = 0x7fffffff;
    for (int q = 0; q < nw; ++q) ist = min(ist, first[par][q]);
    if (ist >= N) break;
    // row ist and column ist of G0 for both spins: four independent loads,
    // issued before the accepted site's data is exchanged
    T gr[2] = {(T)0, (T)0}, gc[2] = {(T)0, (T)0};
    if (own) {
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        gr[sp] = G[sp][(long)ist * N + j];
        gc[sp] = G[sp][(long)j * N + ist];
      }
    }
    if (j == ist) {
      const double du = hj > 0 ? a.dlt_up_p : a.dlt_up_m;
      const double dd = hj > 0 ? a.dlt_dn_p : a.dlt_dn_m;
      const double Ru = 1.0 + (1.0 - d[0]) * du, Rd = 1.0 + (1.0 - d[1]) * dd;
      bF[par][0] = du / Ru;
      bF[par][1] = dd / Rd;
#pragma unroll
      for (int s = 0; s < KM; ++s) {
        bX[par][0][s] = xs[0][s]; bY[par][0][s] = ys[0][s];
        bX[par][1][s] = xs[1][s]; bY[par][1][s] = ys[1][s];
      }
      s_R[s_acc] = Ru * Rd;
      s_acc += 1;
      hj = -hj;
      hl[j] = (int8_t)hj;
      mine = true;
    }
    __syncthreads();
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      T cv = gc[sp], rv = gr[sp];
#pragma unroll
      for (int s = 0; s < KM; ++s) {
        cv -= xs[sp][s] * bY[par][sp][s];
        rv -= bX[par][sp][s] * ys[sp][s];
      }
      const T xn = (T)bF[par][sp] * ((j == ist ? (T)1 : (T)0) - cv);
      const T yn = own ? rv : (T)0;
      const T xv = own ? xn : (T)0;
#pragma unroll
      for (int s = 0; s < KM; ++s)
        if (s == m) { xs[sp][s] = xv; ys[sp][s] = yn; }
      d[sp] -= (double)xv * (double)yn;
    }
    ++m;
    pos = ist + 1;
    par ^= 1;
    // No barrier here: the next acceptance writes the other parity's buffers,
    // and the one after can only write these once every thread has passed
    // the next ballot barrier, i.e. finished reading them.
    if (m == a.k) {
      flush_spin<T, S, KM>(G[0], N, a.fb, xs[0], ys[0], Xs, Ys);
      flush_spin<T, S, KM>(G[1], N, a.fb, xs[1], ys[1], Xs, Ys);
#pragma unroll
      for (int s = 0; s < KM; ++s) { xs[0][s] = xs[1][s] = ys[0][s] = ys[1][s] = (T)0; }
      d[0] = own ? (double)G[0][(long)j * N + j] : 0.0;
      d[1] = own ? (double)G[1][(long)j * N + j] : 0.0;
      m = 0;
    }
  }
  if (m > 0) {
    flush_spin<T, S, KM>(G[0], N, a.fb, xs[0], ys[0], Xs, Ys);
    flush_spin<T, S, KM>(G[1], N, a.fb, xs[1], ys[1], Xs, Ys);
  }
  // diagonal factors of the updated slice for the wrap: D = e^{sigma lambda h}
  if (own) {
    S *dv0 = (S *)a.dv + (2L * c) * 2 * N;
    S *dv1 = dv0 + 2 * N;
    const S up = hj > 0 ? (S)a.elam : (S)a.emlam;
    const S dn = hj > 0 ? (S)a.emlam : (S)a.elam;
    dv0[j] = up; dv0[N + j] = dn;      // spin up: D, D^{-1}
    dv1[j] = dn; dv1[N + j] = up;      // spin down
    if (a.trace_mode == 1 && trace_idx >= 0) a.trace[trace_idx] = mine ? 1 : 0;
  }
  __syncthreads();
  // log-weight of the slice's accepted ratios (FP64), and the check that
  // every proposed ratio was positive and finite
  const int nacc = s_acc;
  double lg = 0.0, bad = (double)badj, neg = 0.0, soft = (double)softj;
  for (int q = j; q < nacc; q += blockDim.x) {
    const double R = s_R[q];
    if (!isfinite(R)) bad = 2.0;
    else if (!(R > 0.0)) bad = fmax(bad, 1.0);
    if (R < 0.0) neg += 1.0;
    lg += log(fabs(R));
  }
  lg = block_sum(lg, red);
  bad = block_max(bad, red);
  neg = block_sum(neg, red);
  soft = block_sum(soft, red);
  if (j == 0) {
    ChainStats *st = a.stats + c;
    st->proposals += N;
    st->accepted += nacc;
    st->logw += lg;
    st->negs += (int)neg;
    st->fp32_rejected += (int)soft;
    if (bad > 0.0) atomicOr(a.err, bad > 1.5 ? (1 | 16) : (1 | 32));
  }
}

// ---------------------------------------------------------------------------
// Paired variant for N <= 256: two lanes per site.  Each lane of the pair
// keeps every other delayed pair (pair m lives in half m & 1, slot m >> 1),
// so the X and Y rows, the dot products of an acceptance and the row that
// the accepted site publishes are split in half; the halves of a dot product
// meet through one cross-lane swap.  The decision, the diagonal and every
// value that enters G are the same in both lanes.  Twice the wavefronts also
// double the loads in flight during a flush.

// LDS strides of the paired flush: rows of -X are padded to KM + 2 (FP64) or
// KM + 4 (FP32) elements and rows of Y^T to sites + 16, so that the MFMA
// operand reads (16 rows or columns by 4 k values per instruction) and the
// owners' writes touch distinct banks
template <typename T, int KM> constexpr int pair_xld() { return KM + (sizeof(T) == 8 ? 2 : 4); }
constexpr int PAIR_YPAD = 16;

// Lane layout: the halves of a site sit in alternate rows of 16 lanes (rows 0
// and 2 hold half 0 of 16 consecutive sites, rows 1 and 3 half 1 of the same
// sites), so all lanes of a row need the same elements of the accepted site's
// vectors: each lane reads one of them from LDS and the dot products take
// them by DPP row broadcast, a sixteenth of the LDS data of a broadcast read.
struct PairLanes {
  static constexpr unsigned long long half0 = 0x0000FFFF0000FFFFull;   // lanes of half 0
  static __device__ __forceinline__ int site(int t) { return (t >> 6) * 32 + ((t >> 5) & 1) * 16 + (t & 15); }
  static __device__ __forceinline__ int half(int t) { return (t >> 4) & 1; }
  static __device__ __forceinline__ int site_in_wave(int lane) { return (lane >> 5) * 16 + (lane & 15); }
};

// value held by the other lane of the site (lane ^ 16): swizzle swapping the
// two rows of each 32-lane half
__device__ __forceinline__ double pair_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One step q of the four dot products of an acceptance (column and row, both
// spins): acc += (lane q of the row's v) * x, with the broadcast taken by the
// FMA itself (DPP row_newbcast on its first source).  Inline assembly because
// the compiler emits a separate DPP move per broadcast; the leading s_nop
// gives the two wait states a DPP read needs after a vector-ALU write, and
// each accumulator is written once per step, three instructions before the
// next step reads it.  Every lane of the wavefront must be active.
template <int Q>
__device__ __forceinline__ void row_fmac4(double &c0, double &c1, double &r0, double &r1, double vy0, double vy1,
                                          double vx0, double vx1, double x0, double x1, double y0, double y1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %5, %9 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %6, %10 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %7, %11 row_newbcast:%c12 row_mask:0xf bank_mask:0xf"
      : "+v"(c0), "+v"(c1), "+v"(r0), "+v"(r1)
      : "v"(vy0), "v"(vy1), "v"(vx0), "v"(vx1), "v"(x0), "v"(x1), "v"(y0), "v"(y1), "n"(Q));
}
// c_s = sum_q xs_s[q] vy_s[q], r_s = sum_q vx_s[q] ys_s[q] (s = both spins),
// accumulated in q order, with vy_s[q], vx_s[q] held by lane q of the row
template <typename T, int H, int... Q>
__device__ __forceinline__ void row_dots(T (&c)[2], T (&r)[2], const T (&vy)[2], const T (&vx)[2], const T (&x)[2][H],
                                         const T (&y)[2][H], std::integer_sequence<int, Q...>) {
  (row_fmac4<Q>(c[0], c[1], r[0], r[1], vy[0], vy[1], vx[0], vx[1], x[0][Q], x[1][Q], y[0][Q], y[1][Q]), ...);
}

// G0 <- G0 - X Y^T for one spin with the pairs split over the two lanes of
// each site (same MFMA scheme as flush_spin).
template <typename T, typename S, int KM>
__device__ void flush_pairs(S *G, int N, int fb, int ldy, const T (&xs)[KM / 2], const T (&ys)[KM / 2], T *Xs,
                            T *Ys) {
  // tiles per wavefront: two batches of TP tiles alternate, the next batch's
  // G tiles loading while the current batch runs its MFMAs (with FP64 MFMA
  // at a quarter of a 16x16x4 block per 16 cycles, the flush is bound by the
  // matrix core once the loads are hidden); 2 x 2 FP64 or 2 x 4 FP32 tiles
  // keep the register budget of 2 waves per SIMD next to the X, Y halves
  constexpr int H = KM / 2, TP = sizeof(T) == 8 ? 2 : 4, XLD = pair_xld<T, KM>();
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
  const int j = PairLanes::site(t), hf = PairLanes::half(t);
  const int l16 = lane & 15, lq = lane >> 4;
  const bool own = j < N;
#pragma unroll
  for (int q = 0; q < H; ++q) Ys[(2 * q + hf) * ldy + j] = own ? ys[q] : (T)0;
  typedef typename Mfma<T>::acc_t acc_t;
  const int ctiles = (N + 15) >> 4;
  for (int i0 = 0; i0 < N; i0 += fb) {
    __syncthreads();
    if (j >= i0 && j < i0 + fb) {
#pragma unroll
      for (int q = 0; q < H; ++q) Xs[(j - i0) * XLD + 2 * q + hf] = own ? -xs[q] : (T)0;
    }
    __syncthreads();
    const int nrb = min(fb, N - i0);
    const int ntiles = ((nrb + 15) >> 4) * ctiles;
    // tiles base + nw * b of a batch; elements outside the block (and tiles
    // past ntiles) read a clamped in-range address and keep zero, so every
    // lane issues its loads unconditionally and the wait before a batch's
    // MFMAs leaves the next batch's loads in flight
    auto load = [&](acc_t (&acc)[TP], int base) {
#pragma unroll
      for (int b = 0; b < TP; ++b) {
        const int tile = base + nw * b;
        const int tr = tile / ctiles, tc = tile % ctiles;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + tr * 16 + Mfma<T>::row(lane, r), col = tc * 16 + l16;
          const bool in = tile < ntiles && row < i0 + nrb && col < N;
          const T v = (T)G[(unsigned)(min(row, N - 1) * N + min(col, N - 1))];
          acc[b][r] = in ? v : (T)0;
        }
      }
    };
    // the batch's tiles advance together through k, so each round of LDS
    // operand reads feeds TP independent MFMAs; a tile past ntiles reads the
    // operands of the last tile and is not stored
    auto run = [&](acc_t (&acc)[TP], int base) {
      int tr[TP], tc[TP];
#pragma unroll
      for (int b = 0; b < TP; ++b) {
        const int tile = min(base + nw * b, ntiles - 1);
        tr[b] = tile / ctiles;
        tc[b] = tile % ctiles;
      }
#pragma unroll
      for (int s0 = 0; s0 < KM; s0 += 4) {
        const int s = s0 + lq;
        T av[TP], bv[TP];
#pragma unroll
        for (int b = 0; b < TP; ++b) {
          av[b] = Xs[(tr[b] * 16 + l16) * XLD + s];
          bv[b] = Ys[s * ldy + tc[b] * 16 + l16];
        }
#pragma unroll
        for (int b = 0; b < TP; ++b) acc[b] = Mfma<T>::mac(av[b], bv[b], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < TP; ++b) {
        if (base + nw * b < ntiles) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = i0 + tr[b] * 16 + Mfma<T>::row(lane, r), col = tc[b] * 16 + l16;
            if (row < i0 + nrb && col < N) G[(unsigned)(row * N + col)] = (S)acc[b][r];
          }
        }
      }
    };
    const int step = nw * TP;
    acc_t a0[TP], a1[TP];
    load(a0, w);
    for (int base = w; base < ntiles; base += 2 * step) {
      load(a1, base + step);
      run(a0, base);
      load(a0, base + 2 * step);
      run(a1, base + step);
    }
  }
  __syncthreads();
}

template <typename T, typename S, int KM>
__global__ __launch_bounds__(512) void k_flip_pairs(FlipArgs a) {
  static_assert(KM % 8 == 0, "pairs are split over two lanes and staged in steps of 4");
  constexpr int H = KM / 2;
  extern __shared__ char smem_raw[];
  T *Xs = (T *)smem_raw;                                  // [fb][KM+1]
  T *Ys = Xs + a.fb * pair_xld<T, KM>();                  // [KM][ldy]
  __shared__ int first[2][8];
  __shared__ T bX[2][2][KM], bY[2][2][KM];
  __shared__ double bF[2][2];
  __shared__ double s_R[256];
  __shared__ double red[16];

  const int N = a.N, t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
  typedef PairLanes PL;
  const int j = PL::site(t), hf = PL::half(t);
  const int ldy = (blockDim.x >> 1) + PAIR_YPAD;
  const int c = blockIdx.x;
  const bool own = j < N;
  const long NN = (long)N * N;
  S *G[2] = {(S *)a.G + (2L * c) * NN, (S *)a.G + (2L * c + 1) * NN};
  int8_t *hl = a.h + ((long)c * a.Lam + (a.l - 1)) * N;
  const int64_t sweep = *a.sweep;

  int hj = own ? hl[j] : 1;
  double uj = 2.0;
  bool forced = false;
  long trace_idx = -1;
  if (own && a.trace_mode != 0) {
    const int64_t rel = sweep - *a.trace_base;
    if (rel >= 0 && rel < a.trace_sweeps)
      trace_idx = ((rel * a.chains_total + a.chain0 + c) * (long)a.Lam + (a.l - 1)) * N + j;
  }
  if (own) {
    if (a.trace_mode == 2) {
      if (trace_idx >= 0) forced = a.trace[trace_idx] != 0;
      else if (hf == 0) atomicOr(a.err, 8);   // replay past the supplied history
    } else {
      uj = uniform53(philox_word0((uint64_t)sweep, (uint64_t)(a.l - 1) * N + j, 0, 0, a.seed + (uint64_t)(a.chain0 + c), a.inst));
    }
  }
  T xs[2][H], ys[2][H];
#pragma unroll
  for (int q = 0; q < H; ++q) { xs[0][q] = xs[1][q] = ys[0][q] = ys[1][q] = (T)0; }
  double d[2];
  d[0] = own ? (double)G[0][(long)j * N + j] : 0.0;
  d[1] = own ? (double)G[1][(long)j * N + j] : 0.0;
  bool mine = false;
  __syncthreads();

  int m = 0, pos = 0, par = 0, nacc = 0;   // nacc: acceptances so far, the same in every lane
  int badj = 0;   // 1: ratio <= 0, 2: ratio not finite
  int softj = 0;  // 1: ratio <= 0 in a guarded FP32 slice (rejected, counted)
  for (;;) {
    bool acc = false;
    if (own && j >= pos) {
      const double du = hj > 0 ? a.dlt_up_p : a.dlt_up_m;
      const double dd = hj > 0 ? a.dlt_dn_p : a.dlt_dn_m;
      const double R = (1.0 + (1.0 - d[0]) * du) * (1.0 + (1.0 - d[1]) * dd);
      acc = (a.trace_mode == 2) ? forced : (uj < R);
      // the last evaluation is the site's proposal: every weight of eq. (3)
      // is positive at half filling, so a ratio that is not a finite positive
      // number is an error whether or not it is accepted
      softj = (a.fp32_guard && isfinite(R) && !(R > 0.0)) ? 1 : 0;
      badj = softj ? 0 : (!isfinite(R) ? 2 : (R > 0.0 ? 0 : 1));
    }
    // both lanes of a site decide alike: look at the lanes of half 0
    const unsigned long long bal = __ballot(acc) & PL::half0;
    if (lane == 0) first[par][w] = bal ? (w * 32 + PL::site_in_wave(__ffsll((long long)bal) - 1)) : 0x7fffffff;
    __syncthreads();
    int ist = 0x7fffffff;
    for (int q = 0; q < nw; ++q) ist = min(ist, first[par][q]);
    if (ist >= N) break;
    T gr[2] = {(T)0, (T)0}, gc[2] = {(T)0, (T)0};
    if (own) {
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        gr[sp] = G[sp][(long)ist * N + j];
        gc[sp] = G[sp][(long)j * N + ist];
      }
    }
    if (j == ist) {
      const double du = hj > 0 ? a.dlt_up_p : a.dlt_up_m;
      const double dd = hj > 0 ? a.dlt_dn_p : a.dlt_dn_m;
      const double Ru = 1.0 + (1.0 - d[0]) * du, Rd = 1.0 + (1.0 - d[1]) * dd;
#pragma unroll
      for (int q = 0; q < H; ++q) {
        bX[par][0][hf * H + q] = xs[0][q]; bY[par][0][hf * H + q] = ys[0][q];
        bX[par][1][hf * H + q] = xs[1][q]; bY[par][1][hf * H + q] = ys[1][q];
      }
      if (hf == 0) {
        bF[par][0] = du / Ru;
        bF[par][1] = dd / Rd;
        s_R[nacc] = Ru * Rd;
        hl[j] = (int8_t)(-hj);
      }
      hj = -hj;
      mine = true;
    }
    __syncthreads();
    const int slot = m >> 1, mine_half = m & 1;
    // the four dot products (column and row, both spins) run as independent
    // chains over this lane's half of the pairs, in pair order, then the two
    // halves meet
    T pc[2] = {(T)0, (T)0}, pr[2] = {(T)0, (T)0};
    {
      const int e = hf * H + min(lane & 15, H - 1);
      const T vy[2] = {bY[par][0][e], bY[par][1][e]}, vx[2] = {bX[par][0][e], bX[par][1][e]};
      row_dots(pc, pr, vy, vx, xs, ys, std::make_integer_sequence<int, H>());
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      pc[sp] += pair_partner(pc[sp]);
      pr[sp] += pair_partner(pr[sp]);
    }
    T xn[2], yn[2];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const T cv = gc[sp] - pc[sp], rv = gr[sp] - pr[sp];
      xn[sp] = own ? (T)bF[par][sp] * ((j == ist ? (T)1 : (T)0) - cv) : (T)0;
      yn[sp] = own ? rv : (T)0;
      d[sp] -= (double)xn[sp] * (double)yn[sp];
    }
    // store the pair in its slot: a branch on the block-uniform slot, so only
    // that slot's registers are written
    const bool keep = hf == mine_half;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      if (q == slot) {
        asm volatile("" ::: "memory");
        if (keep) { xs[0][q] = xn[0]; ys[0][q] = yn[0]; xs[1][q] = xn[1]; ys[1][q] = yn[1]; }
      }
    }
    ++m;
    ++nacc;
    pos = ist + 1;
    par ^= 1;
    // no barrier: the next acceptance uses the other parity's buffers (see k_flip)
    if (m == a.k) {
      flush_pairs<T, S, KM>(G[0], N, a.fb, ldy, xs[0], ys[0], Xs, Ys);
      flush_pairs<T, S, KM>(G[1], N, a.fb, ldy, xs[1], ys[1], Xs, Ys);
#pragma unroll
      for (int q = 0; q < H; ++q) { xs[0][q] = xs[1][q] = ys[0][q] = ys[1][q] = (T)0; }
      d[0] = own ? (double)G[0][(long)j * N + j] : 0.0;
      d[1] = own ? (double)G[1][(long)j * N + j] : 0.0;
      m = 0;
    }
  }
  if (m > 0) {
    flush_pairs<T, S, KM>(G[0], N, a.fb, ldy, xs[0], ys[0], Xs, Ys);
    flush_pairs<T, S, KM>(G[1], N, a.fb, ldy, xs[1], ys[1], Xs, Ys);
  }
  if (own && hf == 0) {
    S *dv0 = (S *)a.dv + (2L * c) * 2 * N;
    S *dv1 = dv0 + 2 * N;
    const S up = hj > 0 ? (S)a.elam : (S)a.emlam;
    const S dn = hj > 0 ? (S)a.emlam : (S)a.elam;
    dv0[j] = up; dv0[N + j] = dn;
    dv1[j] = dn; dv1[N + j] = up;
    if (a.trace_mode == 1 && trace_idx >= 0) a.trace[trace_idx] = mine ? 1 : 0;
  }
  __syncthreads();
  double lg = 0.0, bad = (double)badj, neg = 0.0, soft = hf == 0 ? (double)softj : 0.0;   // one count per site
  for (int q = t; q < nacc; q += blockDim.x) {
    const double R = s_R[q];
    if (!isfinite(R)) bad = 2.0;
    else if (!(R > 0.0)) bad = fmax(bad, 1.0);
    if (R < 0.0) neg += 1.0;
    lg += log(fabs(R));
  }
  lg = block_sum(lg, red);
  bad = block_max(bad, red);
  neg = block_sum(neg, red);
  soft = block_sum(soft, red);
  if (t == 0) {
    ChainStats *st = a.stats + c;
    st->proposals += N;
    st->accepted += nacc;
    st->logw += lg;
    st->negs += (int)neg;
    st->fp32_rejected += (int)soft;
    if (bad > 0.0) atomicOr(a.err, bad > 1.5 ? (1 | 16) : (1 | 32));
  }
}

template <typename T, typename S, int KM>
hipError_t launch_pairs(const FlipArgs &a0, hipStream_t s) {
  FlipArgs a = a0;
  const int sites = ((a.N + 31) / 32) * 32;           // 32 sites per wavefront
  const int threads = 2 * sites;
  constexpr int XLD = pair_xld<T, KM>();
  const size_t ybytes = sizeof(T) * (size_t)KM * (sites + PAIR_YPAD);
  const size_t budget = 146 * 1024;
  int fb = 16;
  while (fb < a.N && ybytes + sizeof(T) * (size_t)(fb + 16) * XLD <= budget) fb += 16;
  a.fb = fb;
  const size_t lds = sizeof(T) * (size_t)fb * XLD + ybytes;
  if (threads > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_flip_pairs<T, S, KM>), dim3(a.chains), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <typename T, typename S, int KM>
hipError_t launch_k(const FlipArgs &a0, hipStream_t s) {
  FlipArgs a = a0;
  const int threads = ((a.N + 63) / 64) * 64;
  // rows of X staged per flush block: as many as fit next to Y^T in ~150 KB
  const size_t ybytes = sizeof(T) * (size_t)KM * (threads + 1);
  const size_t budget = 146 * 1024;   // next to ~10 KB of static LDS
  int fb = 16;
  while (fb < a.N && ybytes + sizeof(T) * (size_t)(fb + 16) * (KM + 1) <= budget) fb += 16;
  a.fb = fb;
  const size_t lds = sizeof(T) * (size_t)fb * (KM + 1) + ybytes;
  if (threads <= 256)
    hipLaunchKernelGGL((k_flip<T, S, KM, 256>), dim3(a.chains), dim3(threads), lds, s, a);
  else if (threads <= 512)
    hipLaunchKernelGGL((k_flip<T, S, KM, 512>), dim3(a.chains), dim3(threads), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_t(const FlipArgs &a, hipStream_t s) {
  if (a.k <= 1) return launch_k<T, S, 1>(a, s);
  if (a.N <= 256) {   // two lanes per site
    if (a.k <= 8) return launch_pairs<T, S, 8>(a, s);
    if (a.k <= 16) return launch_pairs<T, S, 16>(a, s);
    if (a.k <= 32) return launch_pairs<T, S, 32>(a, s);
    return hipErrorInvalidValue;
  }
  if (a.k <= 8) return launch_k<T, S, 8>(a, s);
  if (a.k <= 16) return launch_k<T, S, 16>(a, s);
  if (a.k <= 32) return launch_k<T, S, 32>(a, s);
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t flip_slice(const FlipArgs &a, bool fp64, hipStream_t s) {
  // FP64 arithmetic in both cases; G stored in FP64 or FP32
  return fp64 ? launch_t<double, double>(a, s) : launch_t<double, float>(a, s);
}

}  // namespace bss
