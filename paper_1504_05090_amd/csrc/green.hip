// Equal-time Green functions of one field, recomputed from scratch: the
// library's stabilised recomputation (UDV/QR over blocks of n_stab slices, one-
// sided scale-separated inverse) as a standalone call on a device-resident
// field, for both spins at once.
//
//   G_sigma(l) = (I + B_{l-1} .. B_1 B_Lambda .. B_l)^{-1},
//   B^sigma_q = e^{-dtau K} diag(e^{sigma lambda h_q})          (eqs. (2), (3))
//
// The chain is factored from the right in blocks closed after every slice
// that is a multiple of n_stab, after slice Lambda and at the end of the
// chain (the blocks a sweep starting at slice l would use): for each block
// P, X = P U diag(D), X Pi = Q R (Businger-Golub pivot order), U <- Q,
// D <- diag R, V <- D^{-1} R Pi^T V.  Then, with D = D_b D_s split into its
// parts of modulus >= 1 and <= 1,
//   G = (D_b^{-1} U^T + D_s V)^{-1} D_b^{-1} U^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bssqmc.h"
#include "green.h"
#include "kernels.h"

namespace bss {

namespace {

// scratch layout, in doubles from the base (256-byte aligned sections)
struct Plan {
  int L, N, Lam, n_stab, l;
  double lambda;
  size_t Em, Ep, rm, rp, dvD, P, Pw, U[2], D[2], V[2], W1, W2, Tq, Sq, total;
};

size_t up256(size_t doubles) { return (doubles + 31) & ~(size_t)31; }

Plan make_plan(int L, double U, double dtau, double beta, int n_stab, int l) {
  Plan p{};
  p.L = L;
  p.N = L * L;
  p.Lam = (int)std::lround(beta / dtau);
  p.n_stab = std::min(n_stab, p.Lam);
  p.l = l;
  p.lambda = std::acosh(std::exp(0.5 * dtau * U));
  const size_t NN = (size_t)p.N * p.N, mats = 2;
  size_t off = 0;
  auto take = [&](size_t n) { const size_t at = off; off += up256(n); return at; };
  p.Em = take(NN);
  p.Ep = take(NN);
  p.rm = take(p.L);
  p.rp = take(p.L);
  p.dvD = take(mats * p.n_stab * p.N);
  p.P = take(mats * NN);
  p.Pw = take(mats * NN);
  for (int k = 0; k < 2; ++k) {
    p.U[k] = take(mats * NN);
    p.D[k] = take(mats * p.N);
    p.V[k] = take(mats * NN);
  }
  p.W1 = take(mats * NN);
  p.W2 = take(mats * NN);
  p.Tq = take(mats * qr_tsave_doubles(p.N));
  p.Sq = take(mats * qr_scratch_doubles(p.N));
  p.total = off;
  return p;
}

GemmDesc desc(int N) {
  GemmDesc d{};
  d.M = d.N = d.K = N;
  d.batch = 2;
  d.lda = d.ldb = d.ldc = N;
  d.alpha = 1.0;
  d.beta = 0.0;
  return d;
}

}  // namespace

bss_status green_check(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                       const int8_t *field, const double *G_out, size_t *scratch_bytes) {
  if (L < 2 || !(U >= 0.0) || !std::isfinite(U) || !(t >= 0.0) || !std::isfinite(t) || !(beta > 0.0) ||
      !std::isfinite(beta) || !(dtau > 0.0) || !std::isfinite(dtau) || n_stab < 1 || !field || !G_out)
    return BSS_E_INVALID_ARG;
  const double r = beta / dtau, lam = std::round(r);
  if (lam < 1 || std::fabs(r - lam) > 1e-9 * r) return BSS_E_INVALID_ARG;
  if (l < 1 || l > (int)lam) return BSS_E_INVALID_ARG;
  if (L % 2 != 0 || (long)L * L > 512) return BSS_E_UNSUPPORTED;
  if (scratch_bytes) *scratch_bytes = make_plan(L, U, dtau, beta, n_stab, l).total * sizeof(double);
  return BSS_OK;
}

hipError_t green_run(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                     const int8_t *field, double *G_out, double *base, hipStream_t s) {
  const Plan p = make_plan(L, U, dtau, beta, n_stab, l);
  const int N = p.N;
  const long NN = (long)N * N;
  hipError_t e = build_exp(L, t, dtau, base + p.Em, base + p.Ep, nullptr, nullptr, base + p.rm, base + p.rp,
                           nullptr, nullptr, s);
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  double *Em = base + p.Em, *P = base + p.P, *Pw = base + p.Pw, *dvD = base + p.dvD;
  int cur = 0;
  chk(set_identity_udv(base + p.U[0], base + p.D[0], base + p.V[0], 2, N, s));
  // blocks in the order a sweep starting at slice l visits the slices
  int q = l;
  for (int done = 0; done < p.Lam && e == hipSuccess;) {
    int hi = q;
    while (hi % p.n_stab != 0 && hi != p.Lam && done + (hi - q + 1) < p.Lam) ++hi;
    const int nq = hi - q + 1;
    // P = B_hi .. B_q
    chk(slice_scales(field, 1, p.Lam, N, q, hi, std::exp(p.lambda), std::exp(-p.lambda), dvD, s));
    double *bufs[2] = {P, Pw};
    int b = 0;
    chk(scale_columns(Em, dvD, (long)nq * N, bufs[b], 2, N, s));
    for (int k = 1; k < nq; ++k) {
      GemmDesc d = desc(N);
      d.A = Em; d.sA = 0; d.B = bufs[b]; d.sB = NN; d.C = bufs[b ^ 1]; d.sC = NN;
      d.ks = dvD + (size_t)k * N; d.sks = (long)nq * N;
      chk(gemm_f64(d, false, false, s));
      b ^= 1;
    }
    // (U, D, V) <- UDV of P (U D V)
    GemmDesc d = desc(N);
    d.A = bufs[b]; d.sA = NN; d.B = base + p.U[cur]; d.sB = NN; d.C = base + p.W1; d.sC = NN;
    d.cs = base + p.D[cur]; d.scs = N;
    chk(gemm_f64(d, false, false, s));
    chk(qr_udv_blocked(base + p.W1, base + p.Sq, base + p.Tq, base + p.U[cur ^ 1], base + p.D[cur ^ 1],
                       base + p.W2, 2, N, s));
    GemmDesc v = desc(N);
    v.A = base + p.W2; v.sA = NN; v.B = base + p.V[cur]; v.sB = NN; v.C = base + p.V[cur ^ 1]; v.sC = NN;
    chk(gemm_f64(v, false, false, s));
    cur ^= 1;
    done += nq;
    q = hi == p.Lam ? 1 : hi + 1;
  }
  // G = (D_b^{-1} U^T + D_s V)^{-1} D_b^{-1} U^T, solved into G_out
  chk(fresh_prep(base + p.U[cur], base + p.D[cur], base + p.V[cur], base + p.W1, nullptr, nullptr, G_out, 2, N, s));
  chk(lu_solve_blocked(base + p.W1, G_out, 2, N, s));
  return e;
}

}  // namespace bss

extern "C" {

bss_status bss_green_from_field(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                                const int8_t *field, double *G_out, void *stream) {
  size_t bytes = 0;
  const bss_status st = bss::green_check(L, U, t, beta, dtau, n_stab, l, field, G_out, &bytes);
  if (st != BSS_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  double *base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) return BSS_E_OUT_OF_MEMORY;
  hipError_t e = bss::green_run(L, U, t, beta, dtau, n_stab, l, field, G_out, base, s);
  // the scratch is freed once the work on the stream has finished
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(base);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? BSS_OK : BSS_E_DEVICE;
}

}  // extern "C"
