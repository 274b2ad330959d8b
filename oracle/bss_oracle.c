/*
 * bss_oracle.c -- plain FP64 CPU reference of the BSS-QMC sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see bss_oracle.h): used by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * Everything here is written for a reader checking it against the paper and
 * the textbook algorithms, not for speed: dense triple loops, textbook
 * Householder QR with column pivoting, LU with partial pivoting, rank-1
 * Green-function updates applied immediately, and a full recomputation of
 * the stabilised product chain every time a fresh Green function is needed.
 */
#define _POSIX_C_SOURCE 200809L
#include "bss_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, from the published definition (Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
 * two 64x64->128 multiplications, key schedule bumped by the Weyl constants
 * (golden ratio and sqrt(3)-1) between rounds. */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint64_t orc_draw(uint64_t k0, uint64_t k1, uint64_t s, uint64_t pos, uint64_t tag) {
  uint64_t ctr[4] = {s, pos, tag, 0}, key[2] = {k0, k1}, out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[0];
}

/* uniform in [0,1) with 53 random bits */
static double draw_uniform(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------ */
/* dense helpers (row-major n x n) */

static double *mat_new(int n) { return (double *)calloc((size_t)n * n, sizeof(double)); }

static void mat_eye(int n, double *A) {
  memset(A, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = 1.0;
}

/* C = A B (C distinct from A and B) */
static void mat_mul(int n, const double *A, const double *B, double *C) {
  memset(C, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double a = A[(size_t)i * n + k];
      const double *b = B + (size_t)k * n;
      double *c = C + (size_t)i * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
}

static void mat_transpose(int n, const double *A, double *T) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[(size_t)j * n + i] = A[(size_t)i * n + j];
}

/* Solve M X = B by LU with partial pivoting.  M (n x n) and B (n x m) are
 * overwritten (B with X).  logabsdet/sign receive log|det M| and its sign. */
static void lu_solve(int n, double *M, double *B, int m, double *logabsdet, int *sign) {
  double la = 0.0;
  int sg = 1;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(M[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      double v = fabs(M[(size_t)r * n + k]);
      if (v > best) { best = v; p = r; }
    }
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double tmp = M[(size_t)k * n + j]; M[(size_t)k * n + j] = M[(size_t)p * n + j]; M[(size_t)p * n + j] = tmp;
      }
      for (int j = 0; j < m; ++j) {
        double tmp = B[(size_t)k * m + j]; B[(size_t)k * m + j] = B[(size_t)p * m + j]; B[(size_t)p * m + j] = tmp;
      }
      sg = -sg;
    }
    double piv = M[(size_t)k * n + k];
    if (piv < 0) sg = -sg;
    la += log(fabs(piv));
    for (int r = k + 1; r < n; ++r) {
      double f = M[(size_t)r * n + k] / piv;
      M[(size_t)r * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[(size_t)r * n + j] -= f * M[(size_t)k * n + j];
      for (int j = 0; j < m; ++j) B[(size_t)r * m + j] -= f * B[(size_t)k * m + j];
    }
  }
  /* back substitution with the upper factor */
  for (int k = n - 1; k >= 0; --k) {
    double piv = M[(size_t)k * n + k];
    for (int j = 0; j < m; ++j) {
      double s = B[(size_t)k * m + j];
      for (int c = k + 1; c < n; ++c) s -= M[(size_t)k * n + c] * B[(size_t)c * m + j];
      B[(size_t)k * m + j] = s / piv;
    }
  }
  if (logabsdet) *logabsdet = la;
  if (sign) *sign = sg;
}

/* Householder QR with column pivoting (Businger & Golub; Golub & Van Loan,
 * "Matrix Computations", Sec. 5.4.1): A P = Q R.  On return A holds R in its
 * upper triangle (zeros below), Q is formed explicitly, perm[q] is the
 * original index of pivoted column q.  At every step the pivot is the
 * remaining column with the largest norm over the remaining rows (computed
 * afresh, no norm downdating).  Returns det(Q) = +-1. */
static int qr_pivoted(int n, double *A, double *Q, int *perm) {
  double *V = mat_new(n);          /* reflector j stored in column j, rows j.. */
  double *tau = (double *)calloc((size_t)n, sizeof(double));
  int detq = 1;
  for (int j = 0; j < n; ++j) perm[j] = j;
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = -1.0;
    for (int q = j; q < n; ++q) {
      double s = 0.0;
      for (int r = j; r < n; ++r) s += A[(size_t)r * n + q] * A[(size_t)r * n + q];
      if (s > best) { best = s; p = q; }
    }
    if (p != j) {
      for (int r = 0; r < n; ++r) {
        double tmp = A[(size_t)r * n + j]; A[(size_t)r * n + j] = A[(size_t)r * n + p]; A[(size_t)r * n + p] = tmp;
      }
      int tp = perm[j]; perm[j] = perm[p]; perm[p] = tp;
    }
    /* reflector H = I - tau v v^T mapping x = A[j:, j] to alpha e_1 */
    double xn = 0.0;
    for (int r = j; r < n; ++r) xn += A[(size_t)r * n + j] * A[(size_t)r * n + j];
    xn = sqrt(xn);
    double x0 = A[(size_t)j * n + j];
    double alpha = (x0 > 0) ? -xn : xn;
    double vn = 0.0;
    for (int r = j; r < n; ++r) {
      double v = A[(size_t)r * n + j] - (r == j ? alpha : 0.0);
      V[(size_t)r * n + j] = v;
      vn += v * v;
    }
    tau[j] = (vn > 0.0) ? 2.0 / vn : 0.0;
    if (tau[j] != 0.0) detq = -detq;
    A[(size_t)j * n + j] = alpha;
    for (int r = j + 1; r < n; ++r) A[(size_t)r * n + j] = 0.0;
    for (int q = j + 1; q < n; ++q) {
      double w = 0.0;
      for (int r = j; r < n; ++r) w += V[(size_t)r * n + j] * A[(size_t)r * n + q];
      w *= tau[j];
      for (int r = j; r < n; ++r) A[(size_t)r * n + q] -= w * V[(size_t)r * n + j];
    }
  }
  /* Q = H_0 H_1 ... H_{n-1}, accumulated from the right end */
  mat_eye(n, Q);
  for (int j = n - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    for (int q = 0; q < n; ++q) {
      double w = 0.0;
      for (int r = j; r < n; ++r) w += V[(size_t)r * n + j] * Q[(size_t)r * n + q];
      w *= tau[j];
      for (int r = j; r < n; ++r) Q[(size_t)r * n + q] -= w * V[(size_t)r * n + j];
    }
  }
  free(V);
  free(tau);
  return detq;
}

/* ------------------------------------------------------------------------ */
/* UDV factorisation of a product chain (Loh & Gubernatis): X = U D V with U
 * orthogonal, D diagonal carrying the scales, V well conditioned. */
typedef struct {
  int n;
  double *U, *D, *V;
  int detU;
} udv_t;

static void udv_init(udv_t *f, int n) {
  f->n = n;
  f->U = mat_new(n); f->V = mat_new(n);
  f->D = (double *)malloc(sizeof(double) * (size_t)n);
  mat_eye(n, f->U); mat_eye(n, f->V);
  for (int i = 0; i < n; ++i) f->D[i] = 1.0;
  f->detU = 1;
}

static void udv_free(udv_t *f) { free(f->U); free(f->D); free(f->V); }

/* f <- P f :  X = P U D ;  X Pi = Q R ;  U = Q, D = diag R, V = D^{-1} R Pi^T V */
static void udv_push(udv_t *f, const double *P) {
  int n = f->n;
  double *X = mat_new(n), *Q = mat_new(n), *Vn = mat_new(n);
  int *perm = (int *)malloc(sizeof(int) * (size_t)n);
  mat_mul(n, P, f->U, X);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) X[(size_t)i * n + j] *= f->D[j];
  f->detU = qr_pivoted(n, X, Q, perm);
  for (int i = 0; i < n; ++i) {
    double d = X[(size_t)i * n + i];
    for (int q = i; q < n; ++q) {
      double r = X[(size_t)i * n + q] / d;
      const double *vrow = f->V + (size_t)perm[q] * n;
      for (int j = 0; j < n; ++j) Vn[(size_t)i * n + j] += r * vrow[j];
    }
    f->D[i] = d;
  }
  memcpy(f->U, Q, sizeof(double) * (size_t)n * n);
  memcpy(f->V, Vn, sizeof(double) * (size_t)n * n);
  free(X); free(Q); free(Vn); free(perm);
}

/* scale split of a diagonal entry: big part |b| >= 1, small part |s| <= 1 */
static double big_part(double x) { return fabs(x) >= 1.0 ? x : (x >= 0 ? 1.0 : -1.0); }

/* G = (I + U D V)^{-1} = (Db^{-1} U^T + Ds V)^{-1} Db^{-1} U^T */
static void green_from_udv(const udv_t *f, double *G, double *logabsdet, int *sign) {
  int n = f->n;
  double *M = mat_new(n);
  double la = 0.0;
  int sg = f->detU;
  for (int i = 0; i < n; ++i) {
    double db = big_part(f->D[i]);
    double ds = f->D[i] / db;
    la += log(fabs(db));
    if (db < 0) sg = -sg;
    for (int j = 0; j < n; ++j) {
      double ut = f->U[(size_t)j * n + i] / db;        /* (Db^{-1} U^T)_ij */
      M[(size_t)i * n + j] = ut + ds * f->V[(size_t)i * n + j];
      G[(size_t)i * n + j] = ut;
    }
  }
  double lm;
  int sm;
  lu_solve(n, M, G, n, &lm, &sm);
  if (logabsdet) *logabsdet = la + lm;
  if (sign) *sign = sg * sm;
  free(M);
}

/* ------------------------------------------------------------------------ */
/* model */

struct orc_chain {
  int L, N, Lam, n_stab;
  double t, U, beta, dtau, lambda;
  uint64_t k0, k1;
  double *K, *Em, *Ep;
  int8_t *h;
  double *G[2];
  int l;         /* next slice to visit, 1..Lam */
  int64_t s;     /* sweep index */
  orc_stats st;
};

/* eq. (1): nearest-neighbour hopping on the periodic L x L square lattice.
 * For L = 2 both neighbours in a direction are the same site, so the bond is
 * counted twice. */
void orc_hopping(int L, double t, double *K) {
  int N = L * L;
  memset(K, 0, sizeof(double) * (size_t)N * N);
  const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int i = x + L * y;
      for (int d = 0; d < 4; ++d) {
        int xn = (x + dx[d] + L) % L, yn = (y + dy[d] + L) % L;
        K[(size_t)i * N + xn + L * yn] += -t;
      }
    }
}

/* exp(s A): the Taylor series of the exponential, after scaling s A by 2^-j
 * so that its 1-norm is at most 1/2, then squared j times. */
void orc_expm(int n, const double *A, double s, double *out) {
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += fabs(s * A[(size_t)i * n + j]);
    if (c > nrm) nrm = c;
  }
  int sq = 0;
  while (nrm > 0.5) { nrm *= 0.5; ++sq; }
  double scale = s / ldexp(1.0, sq);
  double *B = mat_new(n), *term = mat_new(n), *tmp = mat_new(n);
  for (size_t k = 0; k < (size_t)n * n; ++k) B[k] = scale * A[k];
  mat_eye(n, out);
  mat_eye(n, term);
  for (int k = 1; k <= 60; ++k) {
    mat_mul(n, term, B, tmp);
    double mx = 0.0;
    for (size_t e = 0; e < (size_t)n * n; ++e) {
      term[e] = tmp[e] / k;
      out[e] += term[e];
      if (fabs(term[e]) > mx) mx = fabs(term[e]);
    }
    if (mx < 1e-20) break;
  }
  for (int k = 0; k < sq; ++k) {
    mat_mul(n, out, out, tmp);
    memcpy(out, tmp, sizeof(double) * (size_t)n * n);
  }
  free(B); free(term); free(tmp);
}

/* Hirsch's discrete transformation of the interaction of one Trotter slice
 * (the Ising field of Sec. 2): cosh(lambda) = exp(dtau U / 2). */
double orc_hs_lambda(double U, double dtau) { return acosh(exp(0.5 * dtau * U)); }

static double sigma_of(int spin) { return spin == 0 ? 1.0 : -1.0; }

int orc_N(const orc_chain *c) { return c->N; }
int orc_Lambda(const orc_chain *c) { return c->Lam; }
int orc_slice(const orc_chain *c) { return c->l; }
int64_t orc_sweep_index(const orc_chain *c) { return c->s; }
double orc_lambda(const orc_chain *c) { return c->lambda; }
void orc_get_Em(const orc_chain *c, double *out) { memcpy(out, c->Em, sizeof(double) * (size_t)c->N * c->N); }
void orc_get_Ep(const orc_chain *c, double *out) { memcpy(out, c->Ep, sizeof(double) * (size_t)c->N * c->N); }

/* B^sigma_l = e^{-dtau K} diag(exp(sigma lambda h_l)): kinetic factor on the
 * left, interaction on the right, as in the product of eq. (2). */
void orc_bmat(const orc_chain *c, const int8_t *field, int l, int spin, double *out) {
  int N = c->N;
  double sg = sigma_of(spin);
  for (int i = 0; i < N; ++i)
    for (int m = 0; m < N; ++m)
      out[(size_t)i * N + m] = c->Em[(size_t)i * N + m] * exp(sg * c->lambda * field[(size_t)(l - 1) * N + m]);
}

/* out <- B_q out  (transposed: out <- B_q^T out) */
static void left_mul_b(const orc_chain *c, const int8_t *field, int q, int spin, int transposed, double *P, double *tmp) {
  int N = c->N;
  double *B = mat_new(N);
  orc_bmat(c, field, q, spin, B);
  if (transposed) {
    double *Bt = mat_new(N);
    mat_transpose(N, B, Bt);
    mat_mul(N, Bt, P, tmp);
    free(Bt);
  } else {
    mat_mul(N, B, P, tmp);
  }
  memcpy(P, tmp, sizeof(double) * (size_t)N * N);
  free(B);
}

/* UDV of B_{q_last} ... B_{q_first} over `count` slices starting at slice
 * `first` and moving up cyclically (first, first+1, ..., Lam, 1, ...).  A block
 * is closed after every slice that is a multiple of n_stab, after slice Lam,
 * and at the end of the chain. */
static void chain_up(const orc_chain *c, const int8_t *field, int spin, int first, int count, udv_t *f) {
  int N = c->N;
  udv_init(f, N);
  if (count <= 0) return;
  double *P = mat_new(N), *tmp = mat_new(N);
  mat_eye(N, P);
  for (int step = 0; step < count; ++step) {
    int q = ((first - 1 + step) % c->Lam) + 1;
    left_mul_b(c, field, q, spin, 0, P, tmp);
    if (q % c->n_stab == 0 || q == c->Lam || step == count - 1) {
      udv_push(f, P);
      mat_eye(N, P);
    }
  }
  free(P); free(tmp);
}

/* UDV of the transposed chain B_{lo}^T ... B_{Lam}^T, i.e. the transpose of
 * B_Lam ... B_lo.  Slices are taken from Lam downwards; a block is closed
 * after a slice q with (q-1) a multiple of n_stab and at the end. */
static void chain_down_T(const orc_chain *c, const int8_t *field, int spin, int lo, udv_t *f) {
  int N = c->N;
  udv_init(f, N);
  if (lo > c->Lam) return;
  double *P = mat_new(N), *tmp = mat_new(N);
  mat_eye(N, P);
  for (int q = c->Lam; q >= lo; --q) {
    left_mul_b(c, field, q, spin, 1, P, tmp);
    if ((q - 1) % c->n_stab == 0 || q == lo) {
      udv_push(f, P);
      mat_eye(N, P);
    }
  }
  free(P); free(tmp);
}

/* G at the start of slice l:  (I + B_{l-1} ... B_1 B_Lam ... B_l)^{-1} */
void orc_fresh_green(const orc_chain *c, const int8_t *field, int l, int spin, double *out) {
  udv_t f;
  chain_up(c, field, spin, l, c->Lam, &f);
  green_from_udv(&f, out, NULL, NULL);
  udv_free(&f);
}

/* eq. (3): det M_sigma with M_sigma = I + B_Lam ... B_1 */
void orc_log_det_M(const orc_chain *c, const int8_t *field, int spin, double *logabs, int *sign) {
  udv_t f;
  double *G = mat_new(c->N);
  chain_up(c, field, spin, 1, c->Lam, &f);
  green_from_udv(&f, G, logabs, sign);
  udv_free(&f);
  free(G);
}

/* G(tau_l, 0) = [ (B_l..B_1)^{-1} + B_Lam..B_{l+1} ]^{-1}
 * With A = B_l..B_1 = Ua Da Va and (B_Lam..B_{l+1})^T = Ub Db Vb:
 *   G = Ub Fb^{-1} Y^{-1} Eb^{-1} Va,
 *   Y = Es (Ua^T Ub) Fb^{-1} + Eb^{-1} (Va Vb^T) Fs,
 * where E = Da^{-1} = Eb Es and F = Db = Fb Fs are split into big (|.|>=1)
 * and small (|.|<=1) parts, so every factor in Y is bounded. */
void orc_gtau0(const orc_chain *c, const int8_t *field, int l, int spin, double *out) {
  int N = c->N;
  udv_t a, b;
  chain_up(c, field, spin, 1, l, &a);
  chain_down_T(c, field, spin, l + 1, &b);
  double *W = mat_new(N), *Vv = mat_new(N), *UaT = mat_new(N), *VbT = mat_new(N);
  double *Y = mat_new(N), *Z = mat_new(N);
  mat_transpose(N, a.U, UaT);
  mat_transpose(N, b.V, VbT);
  mat_mul(N, UaT, b.U, W);
  mat_mul(N, a.V, VbT, Vv);
  for (int i = 0; i < N; ++i) {
    double e = 1.0 / a.D[i];
    double eb = big_part(e), es = e / eb;
    for (int j = 0; j < N; ++j) {
      double fb = big_part(b.D[j]), fs = b.D[j] / fb;
      Y[(size_t)i * N + j] = es * W[(size_t)i * N + j] / fb + Vv[(size_t)i * N + j] * fs / eb;
      Z[(size_t)i * N + j] = a.V[(size_t)i * N + j] / eb;
    }
  }
  lu_solve(N, Y, Z, N, NULL, NULL);
  for (int i = 0; i < N; ++i) {
    double fb = big_part(b.D[i]);
    for (int j = 0; j < N; ++j) Z[(size_t)i * N + j] /= fb;
  }
  mat_mul(N, b.U, Z, out);
  free(W); free(Vv); free(UaT); free(VbT); free(Y); free(Z);
  udv_free(&a); udv_free(&b);
}

/* ------------------------------------------------------------------------ */
/* chain lifecycle */

orc_chain *orc_create(int L, double U, double t, double beta, double dtau,
                      uint64_t seed, int inst, int chain, int n_stab) {
  if (L < 2 || !(U >= 0) || !(beta > 0) || !(dtau > 0) || n_stab < 1 || inst < 0 || chain < 0) return NULL;
  double ratio = beta / dtau;
  int Lam = (int)llround(ratio);
  if (Lam < 1 || fabs(ratio - Lam) > 1e-9 * ratio) return NULL;
  orc_chain *c = (orc_chain *)calloc(1, sizeof(orc_chain));
  c->L = L; c->N = L * L; c->Lam = Lam; c->n_stab = n_stab;
  c->t = t; c->U = U; c->beta = beta; c->dtau = dtau;
  c->lambda = orc_hs_lambda(U, dtau);
  c->k0 = seed + (uint64_t)chain;
  c->k1 = (uint64_t)inst;
  int N = c->N;
  c->K = mat_new(N); c->Em = mat_new(N); c->Ep = mat_new(N);
  orc_hopping(L, t, c->K);
  orc_expm(N, c->K, -dtau, c->Em);
  orc_expm(N, c->K, +dtau, c->Ep);
  c->h = (int8_t *)malloc((size_t)Lam * N);
  for (int l = 1; l <= Lam; ++l)
    for (int i = 0; i < N; ++i) {
      uint64_t w = orc_draw(c->k0, c->k1, 0, (uint64_t)(l - 1) * N + i, 1);
      c->h[(size_t)(l - 1) * N + i] = ((w >> 63) == 0) ? 1 : -1;
    }
  c->G[0] = mat_new(N); c->G[1] = mat_new(N);
  c->l = 1; c->s = 0;
  c->st.sign = 1;
  for (int sp = 0; sp < 2; ++sp) orc_fresh_green(c, c->h, 1, sp, c->G[sp]);
  return c;
}

void orc_destroy(orc_chain *c) {
  if (!c) return;
  free(c->K); free(c->Em); free(c->Ep); free(c->h); free(c->G[0]); free(c->G[1]);
  free(c);
}

void orc_get_field(const orc_chain *c, int8_t *out) { memcpy(out, c->h, (size_t)c->Lam * c->N); }

void orc_set_field(orc_chain *c, const int8_t *in) {
  memcpy(c->h, in, (size_t)c->Lam * c->N);
  c->l = 1;
  for (int sp = 0; sp < 2; ++sp) orc_fresh_green(c, c->h, 1, sp, c->G[sp]);
}

void orc_get_green(const orc_chain *c, int spin, double *out) {
  memcpy(out, c->G[spin], sizeof(double) * (size_t)c->N * c->N);
}

void orc_set_green(orc_chain *c, int spin, const double *in) {
  memcpy(c->G[spin], in, sizeof(double) * (size_t)c->N * c->N);
}

void orc_get_stats(const orc_chain *c, orc_stats *out) { *out = c->st; }

/* ------------------------------------------------------------------------ */
/* the sweep */

/* Ratio of det M' / det M for flipping h_{l,i}, per spin, from the current
 * equal-time G at the start of slice l (eq. (3) with the flipped field):
 * R_sigma = 1 + (1 - G_ii) Delta_sigma,  Delta_sigma = e^{-2 sigma lambda h} - 1. */
void orc_ratio(const orc_chain *c, int l, int i, double *R_up, double *R_dn) {
  int N = c->N;
  double h = c->h[(size_t)(l - 1) * N + i];
  for (int sp = 0; sp < 2; ++sp) {
    double delta = exp(-2.0 * sigma_of(sp) * c->lambda * h) - 1.0;
    double R = 1.0 + (1.0 - c->G[sp][(size_t)i * N + i]) * delta;
    if (sp == 0) *R_up = R; else *R_dn = R;
  }
}

/* Sherman-Morrison update after accepting the flip of h_{l,i}:
 * G <- G - (Delta/R) (e_i - G e_i)(e_i^T G), then h_{l,i} <- -h_{l,i}. */
void orc_accept_update(orc_chain *c, int l, int i) {
  int N = c->N;
  double h = c->h[(size_t)(l - 1) * N + i];
  double *col = (double *)malloc(sizeof(double) * (size_t)N);
  double *row = (double *)malloc(sizeof(double) * (size_t)N);
  for (int sp = 0; sp < 2; ++sp) {
    double *G = c->G[sp];
    double delta = exp(-2.0 * sigma_of(sp) * c->lambda * h) - 1.0;
    double R = 1.0 + (1.0 - G[(size_t)i * N + i]) * delta;
    double f = delta / R;
    for (int j = 0; j < N; ++j) {
      col[j] = (j == i ? 1.0 : 0.0) - G[(size_t)j * N + i];
      row[j] = G[(size_t)i * N + j];
    }
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) G[(size_t)j * N + k] -= f * col[j] * row[k];
  }
  c->h[(size_t)(l - 1) * N + i] = (int8_t)(-h);
  free(col); free(row);
}

/* G <- B_l G B_l^{-1} = e^{-dtau K} (D G D^{-1}) e^{+dtau K}, D = diag(e^{sigma lambda h_l}) */
void orc_wrap(orc_chain *c, int l) {
  int N = c->N;
  double *T = mat_new(N), *S = mat_new(N);
  for (int sp = 0; sp < 2; ++sp) {
    double sg = sigma_of(sp);
    double *G = c->G[sp];
    for (int i = 0; i < N; ++i) {
      double di = exp(sg * c->lambda * c->h[(size_t)(l - 1) * N + i]);
      for (int j = 0; j < N; ++j) {
        double dj = exp(sg * c->lambda * c->h[(size_t)(l - 1) * N + j]);
        S[(size_t)i * N + j] = di * G[(size_t)i * N + j] / dj;
      }
    }
    mat_mul(N, S, c->Ep, T);
    mat_mul(N, c->Em, T, G);
  }
  free(T); free(S);
}

int orc_step_slices(orc_chain *c, int n, const uint8_t *forced, uint8_t *trace) {
  int N = c->N;
  int64_t idx = 0;
  double *Gf = mat_new(N);
  int rc = 0;
  for (int step = 0; step < n && rc == 0; ++step) {
    int l = c->l;
    for (int i = 0; i < N; ++i, ++idx) {
      double Ru, Rd;
      orc_ratio(c, l, i, &Ru, &Rd);
      double R = Ru * Rd;
      /* At half filling every weight of eq. (3) is positive, so a ratio that
       * is not a finite positive number means the Green function is broken:
       * that is an error whether or not the flip is accepted. */
      const int bad = !(R > 0) || !isfinite(R);
      int acc;
      if (forced) {
        acc = forced[idx] != 0;
      } else {
        double u = draw_uniform(orc_draw(c->k0, c->k1, (uint64_t)c->s, (uint64_t)(l - 1) * N + i, 0));
        acc = u < R;   /* Metropolis min(1, R); u == R rejects */
      }
      if (trace) trace[idx] = (uint8_t)acc;
      c->st.proposals++;
      if (acc) {
        c->st.accepted++;
        if (R < 0) c->st.sign = -c->st.sign;   /* sign of the weight, eq. (3) */
      }
      if (bad) { c->st.error = 1; rc = -1; break; }
      if (acc) {
        c->st.logw += log(R);
        orc_accept_update(c, l, i);
      }
    }
    if (rc) break;
    orc_wrap(c, l);
    if (l % c->n_stab == 0 || l == c->Lam) {
      int next = (l == c->Lam) ? 1 : l + 1;
      double drift = 0.0;
      for (int sp = 0; sp < 2; ++sp) {
        orc_fresh_green(c, c->h, next, sp, Gf);
        for (size_t e = 0; e < (size_t)N * N; ++e) {
          double d = fabs(Gf[e] - c->G[sp][e]);
          if (d > drift) drift = d;
        }
        memcpy(c->G[sp], Gf, sizeof(double) * (size_t)N * N);
      }
      c->st.drift_sum += drift;
      c->st.drift_count++;
      if (drift > c->st.drift_max) c->st.drift_max = drift;
    }
    if (l == c->Lam) { c->l = 1; c->s++; } else { c->l = l + 1; }
  }
  free(Gf);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* measurement: double occupancy and the k-resolved G(tau_l, k) (paper sign) */
void orc_measure(const orc_chain *c, double *docc, double *gtk) {
  int N = c->N, L = c->L;
  const double two_pi = 6.283185307179586476925286766559;
  double *Gs[2] = {mat_new(N), mat_new(N)};
  for (int sp = 0; sp < 2; ++sp) orc_fresh_green(c, c->h, 1, sp, Gs[sp]);
  double d = 0.0;
  for (int i = 0; i < N; ++i)
    d += (1.0 - Gs[0][(size_t)i * N + i]) * (1.0 - Gs[1][(size_t)i * N + i]);
  *docc = d / N;
  double *Gt = mat_new(N);
  for (int l = 0; l <= c->Lam; ++l) {
    for (int k = 0; k < N; ++k) gtk[(size_t)l * N + k] = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
      orc_gtau0(c, c->h, l, sp, Gt);
      for (int k = 0; k < N; ++k) {
        double kx = two_pi * (k % L) / L, ky = two_pi * (k / L) / L;
        double s = 0.0;
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) {
            int dx = (i % L) - (j % L), dy = (i / L) - (j / L);
            s += cos(kx * dx + ky * dy) * Gt[(size_t)i * N + j];
          }
        gtk[(size_t)l * N + k] += -0.5 * s / N;
      }
    }
  }
  free(Gt); free(Gs[0]); free(Gs[1]);
}

/* ------------------------------------------------------------------------ */
double orc_run_chains(int L, double U, double t, double beta, double dtau,
                      uint64_t seed, int n_chains, int n_stab, int n_warm, int n_sweeps,
                      int n_threads, int *threads_used) {
  orc_chain **ch = (orc_chain **)calloc((size_t)n_chains, sizeof(orc_chain *));
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int c = 0; c < n_chains; ++c) ch[c] = orc_create(L, U, t, beta, dtau, seed, 0, c, n_stab);
  for (int c = 0; c < n_chains; ++c)
    if (!ch[c]) { for (int d = 0; d < n_chains; ++d) orc_destroy(ch[d]); free(ch); return -1.0; }
  if (n_warm > 0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int c = 0; c < n_chains; ++c) orc_step_slices(ch[c], n_warm * ch[c]->Lam, NULL, NULL);
  }
  int used = 1;
  double t0 = 0.0, t1 = 0.0;
#ifdef _OPENMP
  t0 = omp_get_wtime();
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(static)
    for (int c = 0; c < n_chains; ++c) orc_step_slices(ch[c], n_sweeps * ch[c]->Lam, NULL, NULL);
  }
  t1 = omp_get_wtime();
#else
  {
    struct timespec a, b;
    clock_gettime(CLOCK_MONOTONIC, &a);
    for (int c = 0; c < n_chains; ++c) orc_step_slices(ch[c], n_sweeps * ch[c]->Lam, NULL, NULL);
    clock_gettime(CLOCK_MONOTONIC, &b);
    t0 = 0.0;
    t1 = (b.tv_sec - a.tv_sec) + 1e-9 * (b.tv_nsec - a.tv_nsec);
  }
#endif
  if (threads_used) *threads_used = used;
  for (int c = 0; c < n_chains; ++c) orc_destroy(ch[c]);
  free(ch);
  return t1 - t0;
}
