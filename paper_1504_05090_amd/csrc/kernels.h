// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bss {

// Batched C = alpha * diag(rs) * op(A) diag(ks) op(B) * diag(cs) + beta * C.
// Strides are in elements; a stride of 0 shares one matrix/vector across the batch.
struct GemmDesc {
  int M, N, K, batch;
  const void *A; long lda, sA;
  const void *B; long ldb, sB;
  void *C; long ldc, sC;
  const void *ks; long sks;   // length-K scale of A's columns (nullable)
  const void *rs; long srs;   // length-M scale of the result rows (nullable)
  const void *cs; long scs;   // length-N scale of the result columns (nullable)
  double alpha, beta;
};
hipError_t gemm_f64(const GemmDesc &d, bool ta, bool tb, hipStream_t s);
hipError_t gemm_f32(const GemmDesc &d, bool ta, bool tb, hipStream_t s);

// Per-chain device statistics.
struct ChainStats {
  int64_t proposals, accepted;
  double logw;
  double drift_max, drift_sum;           // max_ij |G_wrapped - G_fresh|
  double rdrift_max, rdrift_sum;         // the same over max(1, max_ij |G_fresh|)
  double rdrift_sweep;                   // largest relative drift of the current sweep
  int64_t drift_count;
  int32_t negs;                          // accepted ratios that were negative
  int32_t fp32_rejected;                 // finite ratios <= 0 met in guarded FP32 slices
};

// Flip phase of one slice for every chain of one instance.
struct FlipArgs {
  int N, Lam, l, k, chains;
  int chain0, chains_total;   // first chain of this launch, chains of the instance
  int fb;               // rows of X staged per flush block (set by the launcher)
  void *G;              // [2*chains][N][N] bulk type
  int8_t *h;            // [chains][Lam][N]
  void *dv;             // out: [2*chains][2][N] bulk type: D_l and D_l^{-1}
  double dlt_up_p, dlt_up_m;   // Delta_up for h = +1 / -1
  double dlt_dn_p, dlt_dn_m;   // Delta_dn for h = +1 / -1
  double elam, emlam;          // e^{lambda}, e^{-lambda}
  uint64_t seed, inst;
  const int64_t *sweep;        // device sweep counter
  int trace_mode;              // 0 none, 1 record, 2 replay
  int fp32_guard;              // FP32-stored G: a finite ratio <= 0 is rejected and
                               // counted (stats fp32_rejected), not an error
  uint8_t *trace;              // [sweeps][chains_total][Lam][N]
  const int64_t *trace_base;   // sweep index of trace entry 0
  int64_t trace_sweeps;        // capacity in sweeps
  ChainStats *stats;
  int *err;
};
hipError_t flip_slice(const FlipArgs &a, bool fp64, hipStream_t s);

// Products with e^{-+dtau K} = R (x) R (R: L x L circulant of the ring
// propagator r, element type of X):
//   hop_left:  Y = (R (x) R) diag(ks) X
//   hop_right: Y = diag(rs) X diag(ks) (R (x) R)
// X, Y: mats N x N row-major matrices (N = L^2, even L <= 22), Y != X.
struct HopDesc {
  int L, mats;
  const void *X; long sX;
  void *Y; long sY;
  const void *r;                 // r(0..L-1)
  const void *ks; long sks;      // scale of X's rows (left) or columns (right), nullable
  const void *rs; long srs;      // scale of X's rows, right action only, nullable
};
hipError_t hop_left(const HopDesc &d, bool f64, hipStream_t s);
hipError_t hop_right(const HopDesc &d, bool f64, hipStream_t s);

// setup: dense e^{-dtau K} and e^{+dtau K} (FP64; Etm / Etp, nullable,
// receive FP32 copies) and their ring factors rm and rp (rtm / rtp,
// nullable: FP32 copies)
hipError_t build_exp(int L, double t, double dtau, double *Em, double *Ep, float *Etm, float *Etp, double *rm,
                     double *rp, float *rtm, float *rtp, hipStream_t s);
hipError_t init_field(int8_t *h, int chains, int Lam, int N, uint64_t seed, uint64_t inst,
                      hipStream_t s);
// out[mat][q - lo][i] = exp(sigma lambda h[chain][q-1][i]), q = lo..hi (FP64)
hipError_t slice_scales(const int8_t *h, int chains, int Lam, int N, int lo, int hi, double elam,
                        double emlam, double *out, hipStream_t s);
// P[mat] = E * diag(d[mat])
hipError_t scale_columns(const double *E, const double *d, long sd, double *P, int mats, int N,
                         hipStream_t s);
hipError_t set_identity_udv(double *U, double *D, double *V, int mats, int N, hipStream_t s);
hipError_t copy_to_bulk(const double *src, void *dst, long n, bool fp64, hipStream_t s);
hipError_t bump_counter(int64_t *ctr, hipStream_t s);

// FP64 stabilisation
// Blocked Householder QR with Businger-Golub pivoting of X (overwritten):
// U = Q, D = diag(R), RP = D^{-1} R Pi^T (so that X = U diag(D) RP).  Tsave
// holds qr_tsave_doubles(N) and Scr qr_scratch_doubles(N) doubles per matrix.
size_t qr_tsave_doubles(int N);
size_t qr_scratch_doubles(int N);
hipError_t qr_udv_blocked(double *X, double *Scr, double *Tsave, double *U, double *D, double *RP, int mats, int N,
                          hipStream_t s);
// M Z = B by blocked LU with partial pivoting (M overwritten by its factors,
// B replaced by Z); N <= 512.
hipError_t lu_solve_blocked(double *M, double *B, int mats, int N, hipStream_t s);
// Middle matrix of the two-sided fresh-G formula and its right-hand side.
hipError_t fresh_prep(const double *UR, const double *DR, const double *VR, double *W1,
                      const double *W2, const double *DL, double *RHS, int mats, int N,
                      hipStream_t s);
// drift = max |G_cmp - Gf| per chain; G_out <- Gf (rounded to G_out's type);
// cmp64 / out64 select FP64 or FP32 for G_cmp / G_out.  count: 0 leaves the
// statistics alone, 1 adds the drift to them, 2 also starts a new sweep's
// rdrift_sweep with it (the sweep's first recomputation).  drift_abort > 0:
// a relative drift above it sets err bit 2.  Each chain is split
// over DRIFT_PARTS workgroups whose maxima go to part (chains * DRIFT_PARTS * 3
// doubles of scratch) before one wavefront per chain reduces them.
constexpr int DRIFT_PARTS = 16;
hipError_t drift_replace(const void *Gcmp, bool cmp64, void *Gout, bool out64, const double *Gf,
                         int chains, int N, double *part, ChainStats *stats, int *err, double drift_abort,
                         int count, hipStream_t s);
// dst <- src between FP64 and FP32 Green-function stacks (n elements)
hipError_t convert_green(const void *src, bool src64, void *dst, bool dst64, long n, hipStream_t s);
// RHS = Ds_R V_R (right-hand side of the time-displaced G(tau_l, 0) system)
hipError_t time_rhs(const double *DR, const double *VR, double *RHS, int mats, int N, hipStream_t s);
// reciprocal of the big parts of D (for the final left product)
hipError_t inv_big(const double *D, double *out, long n, hipStream_t s);

}  // namespace bss
