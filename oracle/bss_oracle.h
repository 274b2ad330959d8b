/*
 * bss_oracle.h -- plain FP64 CPU reference of the BSS-QMC sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library and does not include or link anything from it.
 *
 * What it computes (Rost & Bluemer, "Deciding the fate of the false Mott
 * transition in two dimensions by exact quantum Monte Carlo methods"):
 *   - the half-filled Hubbard model of eq. (1) on an L x L square lattice with
 *     periodic boundaries (Sec. 2),
 *   - its Trotter-decomposed partition function Z_dtau of eq. (2) with
 *     Lambda = beta/dtau slices, kinetic factor on the left of each slice,
 *   - the discrete Hubbard-Stratonovich Ising field h and the determinant form
 *     Z_dtau = sum_h det M_up det M_dn of eq. (3),
 *   - the Monte Carlo summation of eq. (3) (Sec. 2, paragraph after eq. (3)),
 *     producing Green functions G_ij(tau_l) on the grid tau_l in [0, beta].
 * The sweep mechanics (Metropolis ratio, rank-1 Green-function update, wrap,
 * UDV stabilisation) are not spelled out in the paper; they follow the BSS
 * algorithm it cites (Blankenbecler, Scalapino & Sugar 1981), Hirsch's
 * discrete transformation (1983) and the Loh-Gubernatis UDV scheme (1992).
 *
 * Conventions: site i = x + L*y; matrices are row-major N x N doubles;
 * internal Green functions use G = <c c^dagger> (positive); reported G(tau)
 * carries the paper's sign G(tau) = -<T c(tau) c^dagger(0)> (eq. (4)).
 */
#ifndef BSS_ORACLE_H
#define BSS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based generator: Philox4x64-10 (Salmon et al., SC'11) ---- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* word 0 of Philox(key=(k0,k1), ctr=(s,pos,tag,0)) */
uint64_t orc_draw(uint64_t k0, uint64_t k1, uint64_t s, uint64_t pos, uint64_t tag);

/* ---- model pieces ---- */
/* hopping matrix K_ij = -t * (number of nearest-neighbour bonds i-j), PBC */
void orc_hopping(int L, double t, double *K /* N*N */);
/* out = exp(s * A) for a square matrix A (Taylor series + scaling/squaring) */
void orc_expm(int n, const double *A, double s, double *out);
/* lambda with cosh(lambda) = exp(dtau*U/2) */
double orc_hs_lambda(double U, double dtau);

typedef struct orc_chain orc_chain;

/* A chain of instance `inst`, chain index `chain`: RNG key = (seed+chain, inst).
 * The field is drawn from the generator (tag 1) and G(tau=0) is computed fresh.
 * Returns NULL on invalid arguments. */
orc_chain *orc_create(int L, double U, double t, double beta, double dtau,
                      uint64_t seed, int inst, int chain, int n_stab);
void orc_destroy(orc_chain *c);

int orc_N(const orc_chain *c);
int orc_Lambda(const orc_chain *c);
int orc_slice(const orc_chain *c);        /* next slice to visit, 1..Lambda */
int64_t orc_sweep_index(const orc_chain *c);
double orc_lambda(const orc_chain *c);
void orc_get_Em(const orc_chain *c, double *out);  /* e^{-dtau K} */
void orc_get_Ep(const orc_chain *c, double *out);  /* e^{+dtau K} */

void orc_get_field(const orc_chain *c, int8_t *out /* Lambda*N, [l][i] */);
/* replace the field, reset to slice 1 and recompute G(tau=0) from scratch */
void orc_set_field(orc_chain *c, const int8_t *in);
/* current Green function of spin (0 = up, 1 = down), positive convention */
void orc_get_green(const orc_chain *c, int spin, double *out);
/* overwrite the current Green function (used to test one update step) */
void orc_set_green(orc_chain *c, int spin, const double *in);

/* Advance n slices.  forced != NULL: accept bits (one byte per proposal, in
 * visiting order) replace the Metropolis test.  trace != NULL: the accept
 * decisions taken are written there (one byte per proposal).
 * Returns 0, or -1 if a proposal's ratio R = R_up R_dn was non-finite or
 * non-positive (accepted or not); the chain then stops at that proposal with
 * its error flag set. */
int orc_step_slices(orc_chain *c, int n, const uint8_t *forced, uint8_t *trace);

/* single pieces of the sweep, exposed for the unit tests */
void orc_ratio(const orc_chain *c, int l, int i, double *R_up, double *R_dn);
void orc_accept_update(orc_chain *c, int l, int i);   /* flips h and updates G */
void orc_wrap(orc_chain *c, int l);                    /* G <- B_l G B_l^{-1}   */

/* ---- pure functions of a field ---- */
/* B^sigma_l = e^{-dtau K} diag(e^{sigma lambda h_l}) */
void orc_bmat(const orc_chain *c, const int8_t *field, int l, int spin, double *out);
/* equal-time G at the start of slice l (1..Lambda): (I + B_{l-1}..B_1 B_Lam..B_l)^{-1} */
void orc_fresh_green(const orc_chain *c, const int8_t *field, int l, int spin, double *out);
/* log|det(I + B_Lam...B_1)| and its sign for one spin */
void orc_log_det_M(const orc_chain *c, const int8_t *field, int spin, double *logabs, int *sign);
/* time-displaced G(tau_l, 0) = B_l..B_1 G(0), l = 0..Lambda, positive convention */
void orc_gtau0(const orc_chain *c, const int8_t *field, int l, int spin, double *out);

/* measurement from the current field (call at a sweep boundary):
 * docc = (1/N) sum_i (1-G_up,ii)(1-G_dn,ii);  gtk[(l)*N + k], l = 0..Lambda,
 * k = mx + L*my, with the paper's sign. */
void orc_measure(const orc_chain *c, double *docc, double *gtk);

typedef struct {
  int64_t proposals, accepted;
  double drift_max, drift_sum;
  int64_t drift_count;
  double logw;          /* running sum of log R over accepted flips */
  int sign;             /* running product of sgn R over accepted flips (a
                           negative ratio is also an error, so it stays +1
                           on a healthy chain) */
  int error;            /* nonzero after a numerical failure */
} orc_stats;
void orc_get_stats(const orc_chain *c, orc_stats *out);

/* CPU baseline: run n_chains chains of one instance for n_warm untimed and
 * then n_sweeps timed sweeps with OpenMP over chains (one chain per thread).
 * Returns the seconds of the timed sweeps; *threads_used receives the thread
 * count. */
double orc_run_chains(int L, double U, double t, double beta, double dtau,
                      uint64_t seed, int n_chains, int n_stab, int n_warm, int n_sweeps,
                      int n_threads, int *threads_used);

#ifdef __cplusplus
}
#endif
#endif
