/*
 * bssqmc.h -- C ABI of the MI355X (gfx950) BSS-QMC sweep library.
 *
 * The library samples the discrete Hubbard-Stratonovich Ising field h of the
 * Trotter-decomposed partition function of the half-filled Hubbard model,
 *   Z_dtau = sum_h det M_up[h] det M_dn[h]                  (paper, eq. (3))
 * with M_sigma = I + B^sigma_Lambda ... B^sigma_1,
 *   B^sigma_l = e^{-dtau K} diag(e^{sigma lambda h_{l,i}}),  cosh(lambda) = e^{dtau U/2},
 * for H = -t sum_<ij>,sigma c^+_i c_j + U sum_i (n_up - 1/2)(n_dn - 1/2)
 * (eq. (1)) on an L x L square lattice with periodic boundaries (Sec. 2),
 * Lambda = beta/dtau slices (eq. (2)).  The Monte Carlo summation of eq. (3)
 * yields the Green functions G_ij(tau_l) on the grid tau_l = l dtau in
 * [0, beta] (Sec. 2, paragraph after eq. (3)); the library reports their
 * momentum-resolved form and the double occupancy.
 *
 * One sweep visits l = 1..Lambda, i = 0..N-1 (N = L^2) in this fixed order;
 * per proposal it forms the determinant ratio R = R_up R_dn with
 * R_sigma = 1 + (1 - G_sigma,ii)(e^{-2 sigma lambda h_{l,i}} - 1) and accepts
 * iff u < R (Metropolis; u from Philox4x64-10 keyed by (seed + chain,
 * instance) at counter (sweep, (l-1) N + i, 0, 0), 53-bit uniform of word 0).
 * Accepted flips update G by Sherman-Morrison, delayed to rank k; after each
 * slice G is wrapped, G <- B_l G B_l^{-1}; every n_stab slices and at
 * l = Lambda G is recomputed from the B chain by UDV/QR in FP64 and replaces
 * the wrapped G.
 *
 * Conventions
 *   site i = x + L*y; momentum index k = mx + L*my, k = 2 pi (mx, my)/L.
 *   Matrices exchanged through this ABI are row-major FP64 host arrays.
 *   Internal Green functions are G = <c c^+> (positive).  Reported G(tau, k)
 *   has the paper's sign, G(tau) = -<T c(tau) c^+(0)> (eq. (4)).
 *
 * Ownership and threading
 *   The library owns the context and all device state, except an optional
 *   caller-provided workspace (bss_options.workspace), which must stay alive
 *   until bss_destroy.  All other pointer arguments are caller-owned HOST
 *   buffers.  bss_sweep / bss_step_slices are asynchronous on the context's
 *   stream; every bss_get_* / bss_measure_* call synchronises it.  Calls on
 *   one context must be serialised by the caller.
 *
 * Errors
 *   Every call returns a bss_status; nothing throws or aborts across the ABI.
 *   A numerical failure poisons the context: the call that detects it
 *   returns BSS_E_NUMERICAL and later calls return BSS_E_STATE.  Failures are
 *   a proposal whose ratio R is not a finite positive number (accepted or
 *   not: every weight of eq. (3) is positive at half filling), a non-finite
 *   wrapped or recomputed Green function, and a relative wrap drift above
 *   bss_options.drift_abort.  Since sweeps are asynchronous, a failure inside
 *   a sweep is reported by the next synchronising call.
 */
#ifndef BSSQMC_H
#define BSSQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BSS_OK = 0,
  BSS_E_INVALID_ARG = 1,   /* argument out of range or inconsistent             */
  BSS_E_UNSUPPORTED = 2,   /* valid physics the library does not run (odd L ...) */
  BSS_E_OUT_OF_MEMORY = 3, /* device allocation failed or workspace too small    */
  BSS_E_DEVICE = 4,        /* HIP runtime error                                  */
  BSS_E_NUMERICAL = 5,     /* non-finite / non-positive ratio, drift above limit */
  BSS_E_STATE = 6          /* context poisoned, or call not valid in this state  */
} bss_status;

typedef enum {
  BSS_PREC_FP64 = 0,  /* every step in FP64                                        */
  BSS_PREC_MIXED = 1  /* the last fp32_slices slices of every stabilisation block
                         run in FP32 (G, flips, delayed updates and wraps on FP32
                         MFMA with FP32 accumulation), the others in FP64; ratios,
                         UDV/QR and recomputation are always FP64.  An FP32
                         rounding error made s wraps before a recomputation is
                         amplified by those s wraps (roughly e^{2 lambda} each), so
                         FP32 is placed where few wraps follow.                   */
} bss_precision;

/* bss_options.flags */
#define BSS_FLAG_RECORD_TRACE 0x1u /* record accept decisions (see bss_get_trace)     */
#define BSS_FLAG_REPLAY_TRACE 0x2u /* take accept decisions from bss_set_trace        */
#define BSS_FLAG_NO_GRAPH 0x4u     /* bss_sweep launches kernels directly; by default
                                      it captures one unmeasured sweep into a
                                      hipGraph on first use and replays it (measured
                                      sweeps and PROFILE launch directly)            */
#define BSS_FLAG_PROFILE 0x8u      /* time every kernel launch with HIP events        */
#define BSS_FLAG_KRONECKER_HOPPING 0x10u
                                   /* apply e^{-+dtau K} through its Kronecker factors
                                      in the wraps, the block products and the
                                      G(tau, 0) products: the hopping of eq. (1) on the
                                      periodic square lattice splits into commuting x
                                      and y rings, so e^{-s K} = R (x) R with R the
                                      L x L circulant of the ring propagator.  Same
                                      matrices up to rounding, 4 L^5 instead of 2 L^6
                                      multiply-adds per product, bound by HBM
                                      bandwidth.  Default: dense MFMA GEMMs.          */

typedef struct {
  uint32_t struct_size;  /* sizeof(bss_options)                                    */
  int32_t precision;     /* bss_precision                                          */
  int32_t delay_k;       /* delayed-update rank, 1..32; 0 = automatic              */
  int32_t n_stab;        /* slices between FP64 recomputations; 0 = automatic      */
  void *stream;          /* hipStream_t to run on; NULL = a library-owned stream   */
  void *workspace;       /* optional device memory for all state (caller-owned)    */
  size_t workspace_bytes;
  uint32_t flags;        /* BSS_FLAG_*                                             */
  double drift_abort;    /* poison the context if a relative wrap drift
                            max_ij |G_wrapped - G_fresh| / max(1, max_ij |G_fresh|)
                            exceeds this; 0 = never.  Default 0.1: far above the
                            drift of either precision, far below a chain whose
                            ratios no longer mean anything                        */
  int32_t trace_sweeps;  /* capacity of the record buffer, in sweeps               */
  int32_t fp32_slices;   /* BSS_PREC_MIXED: FP32 slices at the end of each block
                            (values >= n_stab: every slice).  0 = automatic: a
                            drift controller.  Sweeps start with no FP32 slice;
                            after every sweep the library reads the largest
                            relative wrap drift d of each instance's chains in
                            that sweep and moves the next sweep's count by one:
                            down if d > fp32_drift_target / 2, up if
                            d e^{2 lambda} < fp32_drift_target / 2 (one more
                            FP32 slice multiplies the FP32 part of the drift by
                            about e^{2 lambda}), never above the largest s with
                            2^-24 e^{2 lambda s} <= 1e-5 (may be 0 at strong
                            coupling).  While the controller adapts, bss_sweep
                            waits for each sweep's recomputations before issuing
                            the next, and launches its kernels directly (no
                            captured sweep); see fp32_adapt_sweeps.  In these
                            FP32 slices a finite ratio R <= 0 (FP32 rounding of
                            a G whose entries reach 1e2..1e3) is rejected and
                            counted (bss_stats.fp32_rejected) instead of being a
                            numerical failure, and the instance runs in FP64
                            from the next sweep on (bss_stats.fp32_fused).
                            With a fixed count, or when replaying a history,
                            such a ratio stays a failure.  Ignored in FP64 mode. */
  double fp32_drift_target; /* the controller's bound on the relative drift;
                            0 = 1e-3                                              */
  int32_t fp32_adapt_sweeps; /* automatic count only: 0 = the controller adapts
                            after every sweep for the context's lifetime; n > 0 =
                            it adapts after each of the context's first n sweeps
                            and then holds the count it reached (bss_stats.
                            fp32_settled).  Sweeps after that are captured and
                            replayed like those of a fixed count.  The FP32 guard
                            stays on: a finite ratio <= 0 in an FP32 slice is
                            still rejected and counted, and at the start of the
                            next bss_sweep call the instance switches to FP64
                            (bss_stats.fp32_fused) and the context stops
                            capturing (its sweeps launch directly from then on). */
} bss_options;

/* One (L, U, t, beta, dtau) instance with its chains.  delay_k and n_stab,
 * when > 0, set this instance's delay depth (1..32) and block length in
 * place of the options' values (0: the options' value, and when that is 0
 * too the automatic one), so that a batch can run each instance with its own
 * tuned parameters (for instance those bss_autotune found for it). */
typedef struct {
  int32_t L;
  double U, t, beta, dtau;
  uint64_t seed;         /* chain c uses Philox key (seed + c, instance index)     */
  int32_t n_chains;
  int32_t delay_k;       /* 0 or 1..32                                             */
  int32_t n_stab;        /* 0 or >= 1 (clamped to Lambda)                          */
} bss_instance;

typedef struct {
  int64_t sweeps;        /* completed sweeps                                       */
  int64_t proposals;     /* summed over chains                                     */
  int64_t accepted;
  double drift_max;      /* max_ij |G_wrapped - G_fresh| over recomputations       */
  double drift_mean;
  double logw;           /* sum over chains of sum log R over accepted flips       */
  int32_t sign;          /* product of sgn R over accepted flips (a negative ratio
                            is also a numerical failure, so +1 on a healthy run) */
  int32_t n_chains;
  int32_t N, Lambda, delay_k, n_stab;  /* resolved parameters                      */
  int32_t fp32_slices;   /* FP32 slices per block of the next sweep (0 in FP64
                            mode; the controller's current count when automatic) */
  double drift_rel_max;  /* drift over max(1, max_ij |G_fresh|), per recomputation */
  double drift_rel_mean;
  int32_t sweep_graph;   /* 1 once bss_sweep replays a captured hipGraph          */
  int32_t shards;        /* chain groups the instance is split into, each on its
                            own streams (every kernel launch covers one group)  */
  double fp32_fraction;  /* fraction of the slices swept since creation or the
                            last bss_reset_stats that ran in FP32               */
  int64_t fp32_rejected; /* ratios <= 0 rejected in the controller's FP32 slices */
  int32_t fp32_fused;    /* 1 once such a ratio switched the instance to FP64   */
  int32_t fp32_settled;  /* 1 once the controller holds the instance's count
                            (after fp32_adapt_sweeps sweeps)                    */
} bss_stats;

/* Per-kernel launch timing collected under BSS_FLAG_PROFILE. */
typedef struct {
  char name[32];         /* kernel family: flip_f32, flip_f64, wrap_f32, wrap_f64,
                            gemm_f64, qr_udv, lu_solve, elementwise,
                            drift_replace, measure                                */
  int64_t launches;
  double total_ms;       /* summed HIP-event durations                             */
} bss_kernel_time;

/* Fill *opt with defaults (FP64, automatic k and n_stab, library stream). */
void bss_options_default(bss_options *opt);

typedef struct bss_ctx bss_ctx;  /* opaque, owned by the library */

/* Create one instance (eq. (1)-(3) parameters; Lambda = beta/dtau must be an
 * integer within 1e-9 relative).  INVALID_ARG: L < 2, U < 0, t < 0, beta <= 0,
 * dtau <= 0, non-integral beta/dtau, n_chains < 1, bad options, out == NULL.
 * UNSUPPORTED: odd L (periodic odd lattices are not bipartite, so the
 * sign-free property does not hold) or N = L^2 > 512.  The field of chain c is
 * drawn uniformly +-1 from the generator (counter (0, (l-1) N + i, 1, 0),
 * +1 iff bit 63 of word 0 is clear) and G(tau = 0) is computed from scratch.
 * opt may be NULL (defaults).  On success *out receives the context. */
bss_status bss_create(int32_t L, double U, double t, double beta, double dtau, uint64_t seed,
                      int32_t n_chains, const bss_options *opt, bss_ctx **out);

/* Create a batch of n_inst instances sharing one context and one stream; an
 * instance's index is its position in `inst` (it is the second Philox key
 * word).  Same argument rules as bss_create for every instance. */
bss_status bss_create_batch(const bss_instance *inst, int32_t n_inst, const bss_options *opt,
                            bss_ctx **out);

/* Device bytes a workspace must provide for this batch and these options. */
bss_status bss_workspace_size(const bss_instance *inst, int32_t n_inst, const bss_options *opt,
                              size_t *bytes);

/* Run n_sweeps full sweeps of every chain of every instance (asynchronous, on
 * the context's stream).  A sweep is the Monte Carlo step over the Ising field
 * of eq. (3) (paper Sec. 2): for l = 1..Lambda and i = 0..N-1, the proposal
 * h_{l,i} -> -h_{l,i} is accepted iff u < R_up R_dn with R_sigma =
 * 1 + (1 - G_sigma,ii) Delta_sigma; accepted flips update G by delayed
 * Sherman-Morrison; after each slice G <- B_l G B_l^{-1}; after every n_stab
 * slices and at l = Lambda, G is recomputed in FP64 from the UDV-stabilised
 * B chain (G_sigma = M_sigma^{-1}, eq. (3)).  measure != 0: after each sweep
 * accumulate double occupancy, the spin correlation and G(tau_l, k) from the
 * fresh G(tau = 0).  STATE if an instance is not at slice 1.  Failures found
 * on the device (a non-finite or non-positive ratio, a non-finite G, a drift
 * above drift_abort) poison the context; this call or a later one returns
 * NUMERICAL. */
bss_status bss_sweep(bss_ctx *c, int32_t n_sweeps, int32_t measure);

/* Advance every instance by n_slices slices of the sweep of bss_sweep
 * (asynchronous); sweeps may end part-way.  Intended for slice-by-slice
 * checks; no measurement; the same failure behaviour. */
bss_status bss_step_slices(bss_ctx *c, int32_t n_slices);

/* Mean (and standard error, if stderr_out != NULL) of G(tau_l, k), the
 * output the paper's Sec. 2 names (G_ij(tau_l) on the slice grid) with the
 * sign of eq. (4): G(tau_l, k) = -1/2 sum_sigma (1/N) sum_ij
 * cos(k.(r_i - r_j)) <c_i(tau_l) c_j^+(0)>, k = 2 pi (mx, my) / L with
 * index k = mx + L my, over all measured sweeps of instance `inst`:
 * mean[l * N + k], l = 0..Lambda (host arrays of len doubles; stderr_out may
 * be NULL).  G(tau_l, 0) is the stable time-displaced Green function: exact
 * products of B from the recomputed G at block boundaries.  len must equal
 * (Lambda + 1) * N.  The error is over chains (per-chain means) when there
 * are >= 2 chains, else over 16..31 equal bins of one chain.  STATE if nothing
 * was measured; NUMERICAL if the context is poisoned. */
bss_status bss_measure_gtau_k(bss_ctx *c, int32_t inst, double *mean, double *stderr_out,
                              int64_t len);

/* Mean (and standard error; stderr_out may be NULL) of the double occupancy
 * D = (1/N) sum_i <n_i,up n_i,dn> = (1/N) sum_i (1 - G_up,ii)(1 - G_dn,ii)
 * (Wick's theorem for each field), errors as for bss_measure_gtau_k. */
bss_status bss_measure_double_occ(bss_ctx *c, int32_t inst, double *mean, double *stderr_out);

/* Real-space spin correlation of Sec. 4 (Fig. 5), accumulated with the other
 * observables: out[r] = C(r) = (1/N) sum_i <S^z_i S^z_{i+r}>, S^z = (n_up -
 * n_dn)/2, r = dx + L dy with periodic wrap, evaluated per field by Wick's
 * theorem from the fresh G(tau = 0).  len must equal N; mean and stderr_out
 * are host arrays of len doubles (stderr_out may be NULL), errors as for
 * bss_measure_gtau_k.  STATE if nothing was measured.  The correlation length
 * follows from bss_correlation_length. */
bss_status bss_measure_spin_corr(bss_ctx *c, int32_t inst, double *mean, double *stderr_out, int64_t len);

/* Discard accumulated measurements. */
bss_status bss_reset_measurements(bss_ctx *c);

/* Wait until all work enqueued on the context has finished; returns the
 * status of any failure the device flagged meanwhile (as bss_get_* would). */
bss_status bss_synchronize(bss_ctx *c);

/* Zero the per-chain counters behind bss_get_stats (proposals, acceptances,
 * log-weight, drift); the sweep count is kept.  Lets a caller state the drift
 * and acceptance of a stretch of sweeps, e.g. after equilibration. */
bss_status bss_reset_stats(bss_ctx *c);

/* Current equal-time Green function (positive convention) of one chain and
 * spin (0 = up, 1 = down), FP64 row-major N x N, at the current slice
 * position (start of the next slice to visit). */
bss_status bss_get_green(bss_ctx *c, int32_t inst, int32_t chain, int32_t spin, double *out);

/* Ising field of one chain, int8 [Lambda][N]. */
bss_status bss_get_field(bss_ctx *c, int32_t inst, int32_t chain, int8_t *out);

/* Replace the field of one chain (entries must be +-1, else INVALID_ARG).
 * Requires every instance at slice 1; recomputes that chain's stabilisation
 * data and G(tau = 0) from scratch. */
bss_status bss_set_field(bss_ctx *c, int32_t inst, int32_t chain, const int8_t *in);

/* Forced history (requires BSS_FLAG_REPLAY_TRACE): accept decisions for the
 * next n_sweeps sweeps of instance `inst`, one byte per proposal (nonzero =
 * accept), ordered [sweep][chain][l][i].  The decisions replace the
 * Metropolis test; sweeping past the supplied history returns STATE. */
bss_status bss_set_trace(bss_ctx *c, int32_t inst, const uint8_t *accept, int32_t n_sweeps);

/* Recorded decisions (requires BSS_FLAG_RECORD_TRACE) of the first n_sweeps
 * sweeps since creation, same layout as bss_set_trace. */
bss_status bss_get_trace(bss_ctx *c, int32_t inst, uint8_t *accept, int32_t n_sweeps);

/* Statistics of instance `inst` (acceptance, drift, log-weight, sign). */
bss_status bss_get_stats(bss_ctx *c, int32_t inst, bss_stats *out);

/* Checkpoint: with buf == NULL, *bytes receives the size needed; otherwise
 * the fields, sweep counters and measurement accumulators are written to buf
 * (*bytes in: capacity, out: size used).  bss_load restores them into a
 * context created with the same instances and options and recomputes every
 * G from its field, so a resumed run continues the same Markov chain. */
bss_status bss_save(bss_ctx *c, void *buf, size_t *bytes);
bss_status bss_load(bss_ctx *c, const void *buf, size_t bytes);

/* Kernel timings since creation or the last bss_reset_profile (requires
 * BSS_FLAG_PROFILE; synchronises).  Writes up to cap entries; *n_out
 * receives the number of kernel families. */
bss_status bss_get_profile(bss_ctx *c, bss_kernel_time *out, int32_t cap, int32_t *n_out);
bss_status bss_reset_profile(bss_ctx *c);

/* Result of bss_autotune. */
typedef struct {
  int32_t precision;     /* BSS_PREC_MIXED if some FP32 slices passed, else FP64  */
  int32_t delay_k, n_stab, fp32_slices;  /* chosen setting                       */
  int32_t met_bound;     /* 1 if its measured drift is within the bound; 0 if no
                            candidate was (the smallest n_stab tried is returned) */
  int32_t candidates;    /* settings timed                                        */
  double ms_per_sweep;   /* trial time of the chosen setting (all chains)         */
  double drift_rel_max;  /* its relative wrap drift over the trial sweeps         */
} bss_tune_result;

/* Autotuner of the launch parameters of one instance (Sec. 2's BSS-QMC sweep
 * does not fix them; they change cost, not the exact result): chains are
 * equilibrated for warmup_sweeps in FP64 at a short block length, then each
 * candidate (delay_k, n_stab, fp32_slices) is loaded with those fields and
 * timed over trial_sweeps; the fastest whose relative wrap drift (as in
 * bss_stats.drift_rel_max) stays <= drift_bound is returned.  The search
 * takes n_stab in {2, 3, 4, 5, 6, 8, 10, 12, 16, 20} (at most Lambda, and
 * only block lengths whose product of slices has a condition estimate
 * e^{n_stab (2 lambda + 8 t dtau)} <= 1e12, the range where the recomputed G
 * is checked against the exact one to 1e-10) at the automatic delay depth,
 * then delay_k from three depths suited to N, then (precision MIXED)
 * fp32_slices = 1, 2, ... until the bound fails.  The instance's own
 * delay_k and n_stab are ignored.  Other
 * fields of *base (precision, flags other than tracing) are kept.  Allocates
 * and frees its own trial contexts on the current device; synchronous.
 * INVALID_ARG: NULL pointers, drift_bound <= 0, warmup_sweeps < 0,
 * trial_sweeps < 1, or an invalid instance or options. */
bss_status bss_autotune(const bss_instance *inst, const bss_options *base, double drift_bound,
                        int32_t warmup_sweeps, int32_t trial_sweeps, bss_tune_result *out);

/* Equal-time Green functions of both spins at the start of slice l
 * (1..Lambda) for one Ising field, recomputed from scratch exactly as a sweep
 * recomputes them every n_stab slices (eq. (3): G_sigma = M_sigma^{-1} with
 * M_sigma = I + B_{l-1} .. B_1 B_Lambda .. B_l; UDV/QR over blocks of n_stab
 * slices, closed after every multiple of n_stab and after Lambda, then the
 * scale-separated inverse; FP64).  field: DEVICE int8 [Lambda][N] (+-1);
 * G_out: DEVICE FP64 [2][N][N], spin up then down, row-major, positive
 * convention; both caller-owned.  Model arguments as for bss_create.  The
 * call allocates its scratch (about 20 N^2 doubles) with hipMalloc, runs on
 * `stream` (a hipStream_t; NULL: the null stream) and returns after the work
 * has finished and the scratch is freed.  INVALID_ARG: bad model arguments,
 * n_stab < 1, l outside 1..Lambda, NULL pointers; UNSUPPORTED: odd L or
 * N > 512; OUT_OF_MEMORY; DEVICE.  Entries of field other than +-1 give
 * undefined results. */
bss_status bss_green_from_field(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab, int32_t l,
                                const int8_t *field, double *G_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments and errors as bss_green_from_field, but the scratch
 * is a fixed device array of the library (bss_green_from_field_noalloc_limit()
 * bytes, 12 MiB: one 16 x 16 field at any n_stab up to several hundred), held
 * by each device from the first call on it until the process ends.  Nothing
 * is allocated or freed and nothing is synchronised: the call enqueues on
 * `stream` and returns.  All calls on one device share that array, so calls
 * that overlap on one device (different streams or host threads) race; calls
 * in order on one stream are safe.  UNSUPPORTED also when the field's scratch
 * would exceed the limit. */
size_t bss_green_from_field_noalloc_limit(void);
bss_status bss_green_from_field_noalloc(int32_t L, double U, double t, double beta, double dtau, int32_t n_stab,
                                        int32_t l, const int8_t *field, double *G_out, void *stream);

/* Overwrite element (i, j) of the current Green function of one chain and
 * spin (in the precision the current slice holds it) with `value`, e.g. a NaN
 * or a value outside [0, 1] on the diagonal.  For tests of the failure
 * handling above: the next sweep meets the broken G as a numerical failure
 * would arise, and every kernel still runs to its end.  Synchronises.
 * INVALID_ARG: bad instance, chain, spin or indices. */
bss_status bss_debug_set_green(bss_ctx *c, int32_t inst, int32_t chain, int32_t spin, int32_t i, int32_t j,
                               double value);

/* ------------------------------------------------------------------------
 * Analysis of the sweep's output (host code, host buffers, synchronous; no
 * GPU needed).  Readings where the paper is silent: cubic splines with
 * not-a-knot ends; a least-squares polynomial in dtau^2 of order
 * min(2, grids - 1); eq. (5) with e^{+i w_n tau}, w_n = (2n+1) pi / beta (the
 * sign that agrees with eq. (6) under eq. (4)'s convention).  INVALID_ARG for
 * sizes out of range, NULL pointers or non-finite inputs; NUMERICAL when a fit
 * or an inverse does not exist. */

/* Trotter elimination (paper Sec. 3, "Trotter bias" paragraph): the Green
 * functions of n_grids >= 2 slice widths dtau[a] at one beta are aligned on
 * the common grid tau_out[0..n_out) (values in [0, beta]) by cubic splines
 * through their slice grids tau_l = l dtau[a], l = 0..Lambda_a, and
 * extrapolated pointwise to dtau -> 0.  G[a]: (Lambda_a + 1) x n_cols values,
 * row-major [l][col] (e.g. the rows of bss_measure_gtau_k).  out: n_out x
 * n_cols, the constant term of each pointwise fit. */
bss_status bss_trotter_extrapolate(int32_t n_grids, const double *dtau, double beta, const double *const *G,
                                   int32_t n_cols, int32_t n_out, const double *tau_out, double *out);

/* Matsubara transform of eq. (5): G(i w_n), n = 0..n_freq-1, of the cubic
 * spline through (tau[i], G[i]), i = 0..n_tau-1 (tau increasing from 0 to
 * beta), integrated exactly piece by piece.  out: 2 n_freq doubles (re, im). */
bss_status bss_matsubara(int32_t n_tau, const double *tau, const double *G, double beta, int32_t n_freq,
                         double *out_re_im);

/* Dyson equation, eq. (6): Sigma_k(i w_n) = i w_n + mu - eps_k - 1/G_k(i w_n)
 * for n = 0..n_freq-1; G and Sigma as (re, im) pairs. */
bss_status bss_dyson(int32_t n_freq, double beta, double eps_k, double mu, const double *G_re_im,
                     double *sigma_re_im);

/* Finite-size extrapolation (paper Sec. 3, last paragraph): values
 * [n_L][n_vals] (row-major; real and imaginary parts as separate values) of
 * lattices L[0..n_L) (n_L >= 3) fitted against 1/L^2 by least-squares
 * polynomials of first and second order.  value = the average of the two
 * constant terms, err = |linear - quadratic|; lin, quad (nullable) receive
 * the constant terms themselves.  All outputs n_vals doubles. */
bss_status bss_finite_size_extrapolate(int32_t n_L, const int32_t *L, int32_t n_vals, const double *values,
                                       double *value, double *err, double *lin, double *quad);

/* Correlation length (paper Sec. 4, Fig. 5): least-squares fit of
 * log|C(x)| = log A - x / xi over 1 <= x <= L/2, |C(x)| the average of
 * |C(x, 0)| and |C(0, x)| of a spin correlation C[r], r = dx + L dy (as
 * bss_measure_spin_corr reports it).  NUMERICAL if a value is 0 or the fit
 * does not decay.  amplitude is nullable. */
bss_status bss_correlation_length(int32_t L, const double *C, double *xi, double *amplitude);

/* Maximum-entropy spectral function (paper Sec. 3, Trotter-bias paragraph,
 * and eq. (4)), used there only to give back a smooth G(tau) through
 * bss_mem_green.  Readings where the paper is silent: A lives on the
 * increasing grid omega[0..n_omega) with trapezoid weights q_j, so eq. (4)
 * reads G(tau_i) = -sum_j q_j A_j e^{-w_j tau_i} / (1 + e^{-w_j beta});
 * chi^2 = sum_i ((G_i(A) - G[i]) / sigma[i])^2 (one standard error per tau
 * point, no covariance); the entropy is S = sum_j q_j (A_j - m_j -
 * A_j ln(A_j / m_j)) relative to the default model m = model[j] > 0; A
 * minimises chi^2/2 - alpha S.  alpha > 0: that alpha; alpha <= 0: the
 * historic alpha, where chi^2 = n_tau, searched in [1e-8, 1e12].
 * Inputs: n_tau >= 2 points tau[i] in [0, beta] with data G[i] and errors
 * sigma[i] > 0; n_omega >= 2 grid points.  Outputs: A (n_omega doubles);
 * alpha_out, chi2_out (nullable) the alpha used and the chi^2 reached.
 * INVALID_ARG for bad sizes, NULL pointers, non-finite or out-of-range
 * inputs; NUMERICAL if the minimisation does not converge, if A would leave
 * the double range (alpha too small for the data), or if the historic alpha
 * does not exist inside the search range (chi^2 stays above n_tau). */
bss_status bss_mem_spectrum(int32_t n_tau, const double *tau, const double *G, const double *sigma, double beta,
                            int32_t n_omega, const double *omega, const double *model, double alpha, double *A,
                            double *alpha_out, double *chi2_out);

/* eq. (4) on the grid of bss_mem_spectrum: G_out[i] = -sum_j q_j A_j
 * e^{-w_j tau_i} / (1 + e^{-w_j beta}) for n_tau >= 1 points tau[i] in
 * [0, beta]; the smooth G(tau) of a maximum-entropy spectrum. */
bss_status bss_mem_green(double beta, int32_t n_omega, const double *omega, const double *A, int32_t n_tau,
                         const double *tau, double *G_out);

/* Release the context (NULL is allowed). */
void bss_destroy(bss_ctx *c);

const char *bss_status_string(bss_status s);
/* Message of the last failed call on c (valid until the next call on c). */
const char *bss_last_error(const bss_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
