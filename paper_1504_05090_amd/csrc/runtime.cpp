// Host runtime of the BSS-QMC sweep library: argument checking, device
// memory layout, the per-slice launch schedule, stabilisation bookkeeping,
// measurement, trace record/replay, checkpoints and the C ABI of bssqmc.h.
//
// Scheduling.  Device state is organised in shards: contiguous chain ranges
// of one instance (by default all its chains), each with its own pair of HIP
// streams (main, aux).  A sweep issues the shards' launch sequences slice by
// slice in turn, so the instances of a batch run concurrently and small
// instances fill the CUs that a large one leaves idle during its
// latency-bound flip phase.  The left-stack rebuild from a sweep's block
// products runs on the aux stream at the start of the next sweep, under its
// first block of slices, which waits for it only at its first recomputation.  Every
// enqueuing call forks from the context stream and joins back into it, so the
// caller sees a single asynchronous stream.  Sharding changes no result:
// random numbers and the accept history are keyed by the chain's index in its
// instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bssqmc.h"
#include "kernels.h"
#include "measure.h"

using namespace bss;

namespace {

constexpr int NBINS = 32;
constexpr int NMAX = 512;

// ---------------------------------------------------------------------------
// device memory carving: one region (library- or caller-owned), 256-byte
// aligned sub-buffers
struct Carver {
  char *base = nullptr;
  size_t off = 0;
  template <typename T> T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * count;
    return p;
  }
};

// chains [chain0, chain0 + C) of instance `inst`
struct Shard {
  // parameters
  int L = 0, N = 0, Lam = 0, C = 0, mats = 0, k = 1, n_stab = 1, nb = 1;
  int m32 = 0;                           // FP32 slices at the end of each block (mixed mode)
  int m32_max = 0;                       // automatic count, the controller's ceiling
  bool adapt = false;                    // mixed mode, automatic count: adjusted after every sweep
  bool settled = false;                  // the controller's count is held (fp32_adapt_sweeps reached)
  int adapted = 0;                       // sweeps the controller has adjusted the count after
  bool fused = false;                    // an FP32 ratio <= 0 was met: FP64 from then on
  int64_t fp32_rej_seen = 0;             // rejected FP32 ratios already acted on
  int64_t slices_run = 0, fp32_run = 0;  // slices swept since the last statistics reset, in FP32
  int inst = 0, chain0 = 0, Ctot = 0;
  double U = 0, t = 0, beta = 0, dtau = 0, lambda = 0;
  uint64_t seed = 0;
  // device state
  double *Em = nullptr, *Ep = nullptr;   // e^{-dtau K}, e^{+dtau K}
  float *Etm = nullptr, *Etp = nullptr;  // FP32 copies (mixed mode)
  double *rm = nullptr, *rp = nullptr;   // their ring factors (Kronecker hopping)
  float *rtm = nullptr, *rtp = nullptr;  // FP32 copies (mixed mode)
  double *G64 = nullptr;                 // G [2C][N][N] while an FP64 slice is current
  float *G32 = nullptr;                  // G [2C][N][N] while an FP32 slice is current (mixed mode)
  void *Tw = nullptr, *dv = nullptr;     // wrap temporary, slice diagonals: sized for FP64
  int8_t *h = nullptr;
  double *dvD = nullptr;                 // [mats][n_stab][N]
  double *Pc = nullptr, *Pw = nullptr;   // block products [nb][mats][N^2]
  double *RU = nullptr, *RD = nullptr, *RV = nullptr;   // right chain after block b: [nb][...]
  double *LU = nullptr, *LD = nullptr, *LV = nullptr;   // left factors, entry b: (B_Lam..B_{l_b+1})^T
  double *W1 = nullptr, *W2 = nullptr, *W3 = nullptr, *Gf = nullptr, *Gt = nullptr, *invb = nullptr;
  double *dpart = nullptr;               // per-workgroup drift maxima [C][DRIFT_PARTS][3]
  double *Tq = nullptr;                  // compact-WY T factors of the blocked QR
  double *Sq = nullptr;                  // column-swap scratch of the blocked QR
  ChainStats *stats = nullptr;
  int64_t *sweep_ctr = nullptr;
  MeasState ms{};
  // streams and host-side position
  hipStream_t s = nullptr, aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_left = nullptr;
  bool left_pending = false;             // a left rebuild on aux not yet waited for by s
  bool left_stale = false;               // the left factors predate the block products
  bool cur64 = true;                     // G64 (true) or G32 holds the current G
  int slice = 1;
  int64_t sweeps = 0;
};

// one instance as the caller sees it: shards [first, first + count)
struct UInst {
  int first = 0, count = 0, C = 0, N = 0, Lam = 0;
  uint8_t *trace = nullptr;              // [trace_alloc][C][Lam][N]
  int64_t *trace_base = nullptr;         // sweep index of trace entry 0
  int64_t trace_alloc = 0;               // sweeps the trace buffer holds
  int64_t trace_cap = 0;                 // sweeps of the current history window
};

size_t nn(const Shard &I) { return (size_t)I.N * I.N; }

// slice l runs in FP32 iff it is among the last m32 slices of its block
bool fp32_slice(const Shard &I, int l) {
  if (I.m32 <= 0) return false;
  const int end = std::min(((l - 1) / I.n_stab + 1) * I.n_stab, I.Lam);
  return end - l < I.m32;
}

}  // namespace

struct bss_ctx {
  std::vector<Shard> sh;
  std::vector<UInst> ui;
  bss_options opt{};
  bool fp64 = true;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev_fork = nullptr;
  char *mem = nullptr;
  size_t mem_bytes = 0;
  bool own_mem = false;
  int *err = nullptr;
  bool poisoned = false;
  std::string last_error;
  int device = 0;
  // BSS_FLAG_PROFILE: event pairs per kernel family, resolved on demand
  bool profile = false;
  struct Fam {
    const char *name;
    int64_t launches = 0;
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  };
  std::vector<Fam> fam;
  std::vector<hipEvent_t> pool;
  // captured (unmeasured) sweeps, two graphs each, keyed by the FP32 slice
  // counts of the shards they were captured with; replayed by bss_sweep
  // Each captured sweep has event objects of its own (the fork event and each
  // shard's main / rebuild events), used only inside its capture and destroyed
  // after its executable graphs: no event object is shared between a capture
  // and direct launches or another capture.
  struct SweepGraph {
    std::vector<int> key;
    hipGraphExec_t g[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev;   // [2 * shard]: main, rebuild
  };
  std::vector<SweepGraph> gcache;
  bool graphs = false;   // capture and replay sweeps (off: NO_GRAPH, PROFILE, or capture failed)
};

namespace {
enum KFam { F_FLIP32, F_FLIP64, F_WRAP32, F_WRAP64, F_HOP64, F_GEMM64, F_QR_UDV, F_LU_SOLVE, F_ELEM, F_DRIFT,
            F_MEAS, F_COUNT };
const char *const FAM_NAMES[F_COUNT] = {"flip_f32", "flip_f64", "wrap_f32", "wrap_f64", "hop_f64", "gemm_f64",
                                        "qr_udv", "lu_solve", "elementwise", "drift_replace", "measure"};

hipEvent_t take_event(bss_ctx *c) {
  if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// brackets the launches issued in its lifetime with a pair of events
struct Timed {
  bss_ctx *c;
  int fam;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timed(bss_ctx *c_, int f, hipStream_t s_) : c(c_), fam(f), s(s_) {
    // (a failed record surfaces in bss_get_profile's elapsed-time query)
    if (c->profile && (a = take_event(c))) (void)hipEventRecord(a, s);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) { c->pool.push_back(a); return; }
    (void)hipEventRecord(b, s);
    c->fam[fam].pending.push_back({a, b});
  }
};

bss_status fail(bss_ctx *c, bss_status s, const std::string &msg) {
  if (c) c->last_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(ctx, BSS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool valid_instance(const bss_instance &in, std::string &why, bss_status &code) {
  code = BSS_E_INVALID_ARG;
  if (in.L < 2) { why = "L must be >= 2"; return false; }
  if (!(in.U >= 0.0) || !std::isfinite(in.U)) { why = "U must be finite and >= 0"; return false; }
  if (!(in.t >= 0.0) || !std::isfinite(in.t)) { why = "t must be finite and >= 0"; return false; }
  if (!(in.beta > 0.0) || !std::isfinite(in.beta)) { why = "beta must be > 0"; return false; }
  if (!(in.dtau > 0.0) || !std::isfinite(in.dtau)) { why = "dtau must be > 0"; return false; }
  const double r = in.beta / in.dtau;
  const double lam = std::round(r);
  if (lam < 1 || std::fabs(r - lam) > 1e-9 * r) { why = "beta/dtau must be an integer"; return false; }
  if (in.n_chains < 1) { why = "n_chains must be >= 1"; return false; }
  if (in.n_chains > 32767) { why = "n_chains must be <= 32767"; return false; }
  if (in.delay_k < 0 || in.delay_k > 32) { why = "delay_k must be in 0..32"; return false; }
  if (in.n_stab < 0) { why = "n_stab must be >= 0"; return false; }
  code = BSS_E_UNSUPPORTED;
  if (in.L % 2) { why = "odd L is not supported (periodic odd lattices are not bipartite)"; return false; }
  if ((long)in.L * in.L > NMAX) { why = "N = L^2 > 512 is not supported"; return false; }
  return true;
}

// automatic delay depth and stabilisation interval
int auto_k(int N) { return N <= 16 ? 1 : (N <= 64 ? 16 : 32); }
int auto_nstab(double U, double t, double dtau) {
  // keep the plain FP64 block product of n slices well conditioned:
  // cond(B) = e^{2 lambda} cond(e^{-dtau K}) with cond(e^{-dtau K}) = e^{8 t dtau}
  // (hopping spectrum [-4t, 4t]); aim at a product condition of ~1e8
  const double lam = std::acosh(std::exp(0.5 * dtau * U));
  const double per = 2.0 * lam + 8.0 * t * dtau;   // log cond of one slice
  int n = (int)std::floor(std::log(1e8) / std::max(per, 1e-3));
  return std::max(1, std::min(n, 10));
}

// FP32 slices per block in mixed mode when the caller leaves it open: an
// FP32 rounding error (2^-24 relative) made s wraps before a recomputation
// grows by about e^{2 lambda} per wrap (the spread of the slice's diagonal
// factors), so take the largest s with 2^-24 e^{2 lambda s} <= 1e-5, an
// estimate of the mean relative drift the FP32 slices add.
int auto_fp32_slices(double lambda, int n_stab) {
  const double budget = std::log(1e-5 * 16777216.0);
  if (lambda <= 0.0) return n_stab;
  const int s = (int)std::floor(budget / (2.0 * lambda));
  return std::max(0, std::min(s, n_stab));
}

// Shards per instance.  A context of one instance whose sweeps are replayed
// from captured graphs splits its chains into up to four shards of at least
// 32 chains, each on its own streams: the flip kernel of a shard fills only
// as many CUs as it has chains and the QRs are latency-bound, so the shards'
// launches overlap (16 x 16, 128 chains, FP64: 73.9 ms per sweep with one
// shard, 72.3 with two, 71.6 with four).  A context that launches directly
// (the FP32 drift controller, BSS_FLAG_NO_GRAPH, BSS_FLAG_PROFILE) keeps one
// shard: with four, its eight streams share the process's four hardware
// queues, and the sweep took 78 to 104 ms from run to run, against 73 ms with
// one (mixed, the same workload).  A controller context keeps its one shard
// after it settles and its sweeps are captured, so that the held sweeps launch
// the same kernels as the adapting ones.  A batch of several instances already
// overlaps its instances and keeps one shard each.  The environment variable
// BSS_SHARDS = 1..8 overrides, for tuning.
int shard_count(int C, int n_instances, bool direct) {
  int s = n_instances == 1 ? std::min(direct ? 1 : 4, C / 32) : 1;
  if (const char *env = std::getenv("BSS_SHARDS")) {
    const int v = std::atoi(env);
    if (v >= 1 && v <= 8) s = v;
  }
  return std::max(1, std::min(s, C));
}

void layout_shard(Shard &I, bool fp64, Carver &cv) {
  const size_t NN = nn(I), M = (size_t)I.mats;
  I.Em = cv.take<double>(NN);
  I.Ep = cv.take<double>(NN);
  if (!fp64) { I.Etm = cv.take<float>(NN); I.Etp = cv.take<float>(NN); }
  I.rm = cv.take<double>(I.L);
  I.rp = cv.take<double>(I.L);
  if (!fp64) { I.rtm = cv.take<float>(I.L); I.rtp = cv.take<float>(I.L); }
  I.G64 = cv.take<double>(M * NN);
  if (!fp64) I.G32 = cv.take<float>(M * NN);
  I.Tw = cv.take<double>(M * NN);
  I.dv = cv.take<double>(M * 2 * I.N);
  I.h = cv.take<int8_t>((size_t)I.C * I.Lam * I.N);
  I.dvD = cv.take<double>(M * I.n_stab * I.N);
  I.Pc = cv.take<double>((size_t)I.nb * M * NN);
  I.Pw = cv.take<double>(M * NN);
  I.RU = cv.take<double>((size_t)I.nb * M * NN);
  I.RD = cv.take<double>((size_t)I.nb * M * I.N);
  I.RV = cv.take<double>((size_t)I.nb * M * NN);
  I.LU = cv.take<double>((size_t)I.nb * M * NN);
  I.LD = cv.take<double>((size_t)I.nb * M * I.N);
  I.LV = cv.take<double>((size_t)I.nb * M * NN);
  I.W1 = cv.take<double>(M * NN);
  I.W2 = cv.take<double>(M * NN);
  I.W3 = cv.take<double>(M * NN);
  I.Gf = cv.take<double>(M * NN);
  I.Gt = cv.take<double>(M * NN);
  I.invb = cv.take<double>(M * I.N);
  I.dpart = cv.take<double>((size_t)I.C * DRIFT_PARTS * 3);
  I.Tq = cv.take<double>(M * qr_tsave_doubles(I.N));
  I.Sq = cv.take<double>(M * qr_scratch_doubles(I.N));
  I.stats = cv.take<ChainStats>(I.C);
  I.sweep_ctr = cv.take<int64_t>(1);
  I.ms.nbins = NBINS;
  I.ms.nbins_g = I.Ctot == 1 ? NBINS : 1;
  I.ms.glen = (long)(I.Lam + 1) * I.N;
  I.ms.docc = cv.take<double>((size_t)I.C * NBINS);
  I.ms.gk = cv.take<double>((size_t)I.C * I.ms.nbins_g * I.ms.glen);
  I.ms.sclen = I.N;
  I.ms.sc = cv.take<double>((size_t)I.C * I.ms.nbins_g * I.ms.sclen);
  I.ms.count = cv.take<int64_t>(I.C);
  I.ms.binsize = cv.take<int64_t>(I.C);
  I.ms.cur = cv.take<int>(I.C);
}

void layout_inst(UInst &U, Carver &cv, int64_t trace_sweeps, bool tracing) {
  U.trace_alloc = U.trace_cap = tracing ? trace_sweeps : 0;
  U.trace = cv.take<uint8_t>(tracing ? (size_t)trace_sweeps * U.C * U.Lam * U.N : 1);
  U.trace_base = cv.take<int64_t>(1);
}

bool resolve(const bss_instance *in, int n, const bss_options &opt, std::vector<Shard> &out,
             std::vector<UInst> &uis, std::string &why, bss_status &code) {
  out.clear();
  uis.clear();
  for (int i = 0; i < n; ++i) {
    if (!valid_instance(in[i], why, code)) { why = "instance " + std::to_string(i) + ": " + why; return false; }
    Shard I;
    I.L = in[i].L; I.N = I.L * I.L; I.U = in[i].U; I.t = in[i].t; I.beta = in[i].beta; I.dtau = in[i].dtau;
    I.Lam = (int)std::lround(I.beta / I.dtau);
    I.Ctot = in[i].n_chains; I.seed = in[i].seed; I.inst = i;
    I.lambda = std::acosh(std::exp(0.5 * I.dtau * I.U));
    // the instance's own setting, else the options', else automatic
    I.k = in[i].delay_k > 0 ? in[i].delay_k : (opt.delay_k > 0 ? opt.delay_k : auto_k(I.N));
    I.n_stab = in[i].n_stab > 0 ? in[i].n_stab : (opt.n_stab > 0 ? opt.n_stab : auto_nstab(I.U, I.t, I.dtau));
    I.n_stab = std::min(I.n_stab, I.Lam);
    I.nb = (I.Lam + I.n_stab - 1) / I.n_stab;
    if (opt.precision == BSS_PREC_MIXED) {
      if (opt.fp32_slices > 0) {
        I.m32 = I.m32_max = std::min(opt.fp32_slices, I.n_stab);
      } else {
        // automatic: start in FP64, the drift controller raises the count
        I.m32_max = auto_fp32_slices(I.lambda, I.n_stab);
        I.m32 = 0;
        I.adapt = I.m32_max > 0;
      }
    }
    UInst U;
    U.first = (int)out.size();
    U.C = I.Ctot; U.N = I.N; U.Lam = I.Lam;
    const bool direct = I.adapt || (opt.flags & (BSS_FLAG_NO_GRAPH | BSS_FLAG_PROFILE)) != 0;
    U.count = shard_count(I.Ctot, n, direct);
    int c0 = 0;
    for (int s = 0; s < U.count; ++s) {
      Shard J = I;
      J.C = I.Ctot / U.count + (s < I.Ctot % U.count ? 1 : 0);
      J.chain0 = c0;
      J.mats = 2 * J.C;
      c0 += J.C;
      out.push_back(J);
    }
    uis.push_back(U);
  }
  return true;
}

bool check_options(const bss_options *o, std::string &why) {
  if (!o) return true;
  if (o->struct_size != sizeof(bss_options)) { why = "bss_options.struct_size mismatch"; return false; }
  if (o->precision != BSS_PREC_FP64 && o->precision != BSS_PREC_MIXED) { why = "bad precision"; return false; }
  if (o->delay_k < 0 || o->delay_k > 32) { why = "delay_k must be in 0..32"; return false; }
  if (o->n_stab < 0) { why = "n_stab must be >= 0"; return false; }
  if ((o->flags & BSS_FLAG_RECORD_TRACE) && (o->flags & BSS_FLAG_REPLAY_TRACE)) { why = "record and replay are exclusive"; return false; }
  if ((o->flags & BSS_FLAG_RECORD_TRACE) && o->trace_sweeps < 1) { why = "trace_sweeps must be >= 1 to record"; return false; }
  if (o->trace_sweeps < 0) { why = "trace_sweeps must be >= 0"; return false; }
  if (o->fp32_slices < 0) { why = "fp32_slices must be >= 0"; return false; }
  if (!(o->drift_abort >= 0.0)) { why = "drift_abort must be >= 0"; return false; }
  if (!(o->fp32_drift_target >= 0.0)) { why = "fp32_drift_target must be >= 0"; return false; }
  if (o->fp32_adapt_sweeps < 0) { why = "fp32_adapt_sweeps must be >= 0"; return false; }
  return true;
}

// lays the whole context out on `cv` (error word first)
void layout_all(std::vector<Shard> &v, std::vector<UInst> &u, const bss_options &opt, Carver &cv, int **err) {
  int *e = cv.take<int>(4);
  if (err) *err = e;
  const bool tracing = (opt.flags & (BSS_FLAG_RECORD_TRACE | BSS_FLAG_REPLAY_TRACE)) != 0;
  for (auto &I : v) layout_shard(I, opt.precision == BSS_PREC_FP64, cv);
  for (auto &U : u) layout_inst(U, cv, std::max(opt.trace_sweeps, 1), tracing);
}

size_t total_bytes(std::vector<Shard> &v, std::vector<UInst> &u, const bss_options &opt) {
  Carver cv;
  layout_all(v, u, opt, cv, nullptr);
  return cv.off + 256;
}

// ---------------------------------------------------------------------------
// launch schedule of one shard

GemmDesc gemm_desc(int N, int batch) {
  GemmDesc d{};
  d.M = d.N = d.K = N;
  d.batch = batch;
  d.lda = d.ldb = d.ldc = N;
  d.alpha = 1.0;
  d.beta = 0.0;
  return d;
}

struct Exec {
  bss_ctx *c;
  Shard &I;
  const UInst &U;
  hipStream_t s;   // stream the current phase is issued on
  hipError_t e = hipSuccess;
  Exec(bss_ctx *c_, Shard &I_) : c(c_), I(I_), U(c_->ui[I_.inst]), s(I_.s) {}
  void chk(hipError_t x) { if (e == hipSuccess && x != hipSuccess) e = x; }

  size_t NN() const { return nn(I); }
  double *Pc(int b) const { return I.Pc + (size_t)b * I.mats * NN(); }
  double *RU(int b) const { return I.RU + (size_t)b * I.mats * NN(); }
  double *RD(int b) const { return I.RD + (size_t)b * I.mats * I.N; }
  double *RV(int b) const { return I.RV + (size_t)b * I.mats * NN(); }
  double *LU(int b) const { return I.LU + (size_t)b * I.mats * NN(); }
  double *LD(int b) const { return I.LD + (size_t)b * I.mats * I.N; }
  double *LV(int b) const { return I.LV + (size_t)b * I.mats * NN(); }

  bool fp32_at(int l) const { return fp32_slice(I, l); }
  void *Gcur() const { return I.cur64 ? (void *)I.G64 : (void *)I.G32; }
  // the current G in the precision slice l needs (FP64 -> FP32 inside a block)
  void use_precision(int l) {
    const bool want64 = !fp32_at(l);
    if (want64 == I.cur64) return;
    Timed tm(c, F_ELEM, s);
    chk(convert_green(Gcur(), I.cur64, want64 ? (void *)I.G64 : (void *)I.G32, want64, (long)I.mats * NN(), s));
    I.cur64 = want64;
  }
  // fresh G from Gf into the precision of slice `next`, with the drift
  // against the current G recorded when `count`
  void replace(int next, int count, double abort_at) {
    const bool out64 = !fp32_at(next);
    Timed tm(c, F_DRIFT, s);
    chk(drift_replace(Gcur(), I.cur64, out64 ? (void *)I.G64 : (void *)I.G32, out64, I.Gf, I.C, I.N, I.dpart, I.stats,
                      c->err, abort_at, count, s));
    I.cur64 = out64;
  }

  // the main stream waits for an outstanding left rebuild before it touches
  // the left factors, the block products or the QR scratch
  void wait_left() {
    if (!I.left_pending) return;
    chk(hipStreamWaitEvent(I.s, I.ev_left, 0));
    I.left_pending = false;
  }

  void gemm64(const double *A, bool ta, const double *B, bool tb, double *C, long sA, long sB,
              const double *ks = nullptr, long sks = 0, const double *cs = nullptr, long scs = 0) {
    GemmDesc d = gemm_desc(I.N, I.mats);
    d.A = A; d.sA = sA; d.B = B; d.sB = sB; d.C = C; d.sC = (long)NN();
    d.ks = ks; d.sks = sks; d.cs = cs; d.scs = scs;
    Timed tm(c, F_GEMM64, s);
    chk(gemm_f64(d, ta, tb, s));
  }

  bool kron() const { return (c->opt.flags & BSS_FLAG_KRONECKER_HOPPING) != 0; }

  // out = e^{-dtau K} diag(ks) X (FP64), as a dense GEMM or through the
  // Kronecker factors
  void hop64(const double *X, double *out, const double *ks, long sks) {
    if (!kron()) {
      gemm64(I.Em, false, X, false, out, 0, (long)NN(), ks, sks);
      return;
    }
    HopDesc d{};
    d.L = I.L; d.mats = I.mats;
    d.X = X; d.sX = (long)NN(); d.Y = out; d.sY = (long)NN();
    d.r = I.rm; d.ks = ks; d.sks = sks;
    Timed tm(c, F_HOP64, s);
    chk(hop_left(d, true, s));
  }

  // P_b = B_hi ... B_lo (FP64) into Pc(b)
  void block_product(int b) {
    const int lo = b * I.n_stab + 1, hi = std::min((b + 1) * I.n_stab, I.Lam), nq = hi - lo + 1;
    double *bufs[2] = {Pc(b), I.Pw};
    int cur = (nq % 2 == 1) ? 0 : 1;     // so that the last product lands in Pc(b)
    {
      Timed tm(c, F_ELEM, s);
      chk(slice_scales(I.h, I.C, I.Lam, I.N, lo, hi, std::exp(I.lambda), std::exp(-I.lambda), I.dvD, s));
      chk(scale_columns(I.Em, I.dvD, (long)nq * I.N, bufs[cur], I.mats, I.N, s));
    }
    for (int q = 1; q < nq; ++q) {
      hop64(bufs[cur], bufs[cur ^ 1], I.dvD + (size_t)q * I.N, (long)nq * I.N);
      cur ^= 1;
    }
  }

  // (U,D,V)_out = UDV of op(A) (U D V)_in
  void udv_update(const double *A, bool ta, const double *Ui, const double *Di, const double *Vi, double *Uo,
                  double *Do, double *Vo) {
    gemm64(A, ta, Ui, false, I.W1, (long)NN(), (long)NN(), nullptr, 0, Di, I.N);
    {
      Timed tm(c, F_QR_UDV, s);
      chk(qr_udv_blocked(I.W1, I.Sq, I.Tq, Uo, Do, I.W2, I.mats, I.N, s));
    }
    gemm64(I.W2, false, Vi, false, Vo, (long)NN(), (long)NN());
  }

  // G = (I + R L)^{-1} from the right chain after block b and left entry b
  // (none for the last block), into out.  With rhs_v the right-hand side is
  // Ds_R V_R instead, which yields G(tau_{l_b}, 0) (time-displaced).
  void fresh(int b, bool rhs_v, double *out) {
    const bool left = b < I.nb - 1;
    if (left) {
      gemm64(RU(b), true, LU(b), false, I.W1, (long)NN(), (long)NN());
      gemm64(RV(b), false, LV(b), true, I.W2, (long)NN(), (long)NN());
      Timed tm(c, F_ELEM, s);
      chk(fresh_prep(RU(b), RD(b), RV(b), I.W1, I.W2, LD(b), I.W3, I.mats, I.N, s));
    } else {
      Timed tm(c, F_ELEM, s);
      chk(fresh_prep(RU(b), RD(b), RV(b), I.W1, nullptr, nullptr, I.W3, I.mats, I.N, s));
    }
    if (rhs_v) { Timed tm(c, F_ELEM, s); chk(time_rhs(RD(b), RV(b), I.W3, I.mats, I.N, s)); }
    { Timed tm(c, F_LU_SOLVE, s); chk(lu_solve_blocked(I.W1, I.W3, I.mats, I.N, s)); }
    if (left) {
      { Timed tm(c, F_ELEM, s); chk(inv_big(LD(b), I.invb, (long)I.mats * I.N, s)); }
      gemm64(LU(b), false, I.W3, false, out, (long)NN(), (long)NN(), I.invb, I.N);
    } else {
      chk(hipMemcpyAsync(out, I.W3, sizeof(double) * I.mats * NN(), hipMemcpyDeviceToDevice, s));
    }
  }

  void right_update(int b) {
    if (b == 0) {
      chk(set_identity_udv(I.W3, I.invb, I.Gt, I.mats, I.N, s));   // identity U, D, V scratch
      udv_update(Pc(0), false, I.W3, I.invb, I.Gt, RU(0), RD(0), RV(0));
    } else {
      udv_update(Pc(b), false, RU(b - 1), RD(b - 1), RV(b - 1), RU(b), RD(b), RV(b));
    }
  }

  void left_rebuild() {
    const int last = I.nb - 1;
    chk(set_identity_udv(LU(last), LD(last), LV(last), I.mats, I.N, s));
    for (int b = last - 1; b >= 0; --b) udv_update(Pc(b + 1), true, LU(b + 1), LD(b + 1), LV(b + 1), LU(b), LD(b), LV(b));
  }

  // full recomputation from the current field (creation, set_field, load)
  void initialise(bool draw_field) {
    wait_left();
    if (draw_field) chk(init_field(I.h, I.C, I.Lam, I.N, I.seed + (uint64_t)I.chain0, (uint64_t)I.inst, s));
    for (int b = 0; b < I.nb; ++b) {
      block_product(b);
      right_update(b);
    }
    fresh(I.nb - 1, false, I.Gf);
    replace(I.slice, 0, 0.0);
    left_rebuild();
    I.left_stale = false;
  }

  void flip(int l) {
    use_precision(l);
    FlipArgs a{};
    a.N = I.N; a.Lam = I.Lam; a.l = l; a.k = I.k; a.chains = I.C;
    a.chain0 = I.chain0; a.chains_total = I.Ctot;
    a.G = Gcur(); a.h = I.h; a.dv = I.dv;
    a.dlt_up_p = std::exp(-2.0 * I.lambda) - 1.0;   // sigma = +1, h = +1
    a.dlt_up_m = std::exp(2.0 * I.lambda) - 1.0;    // sigma = +1, h = -1
    a.dlt_dn_p = std::exp(2.0 * I.lambda) - 1.0;    // sigma = -1, h = +1
    a.dlt_dn_m = std::exp(-2.0 * I.lambda) - 1.0;   // sigma = -1, h = -1
    a.elam = std::exp(I.lambda); a.emlam = std::exp(-I.lambda);
    a.seed = I.seed; a.inst = (uint64_t)I.inst;
    a.sweep = I.sweep_ctr;
    a.trace_mode = (c->opt.flags & BSS_FLAG_RECORD_TRACE) ? 1 : ((c->opt.flags & BSS_FLAG_REPLAY_TRACE) ? 2 : 0);
    // FP32 slices of the drift controller: a finite ratio <= 0 (FP32 rounding
    // of a G with large entries) is rejected and counted; the controller then
    // runs the instance in FP64
    a.fp32_guard = (!I.cur64 && (I.adapt || I.settled) && a.trace_mode != 2) ? 1 : 0;
    a.trace = U.trace; a.trace_base = U.trace_base; a.trace_sweeps = U.trace_cap;
    a.stats = I.stats; a.err = c->err;
    Timed tm(c, I.cur64 ? F_FLIP64 : F_FLIP32, s);
    chk(flip_slice(a, I.cur64, s));
  }

  // G <- e^{-dtau K} (D G D^{-1}) e^{+dtau K} in the current G's precision
  void wrap() {
    if (!kron()) return wrap_gemm();
    const bool f64 = I.cur64;
    const size_t esz = f64 ? 8 : 4;
    // T = (D G D^{-1}) e^{+dtau K}
    HopDesc d{};
    d.L = I.L; d.mats = I.mats;
    d.X = Gcur(); d.sX = (long)NN(); d.Y = I.Tw; d.sY = (long)NN();
    d.r = f64 ? (const void *)I.rp : (const void *)I.rtp;
    d.rs = I.dv; d.srs = 2L * I.N;
    d.ks = (char *)I.dv + esz * I.N; d.sks = 2L * I.N;
    {
      Timed tm(c, f64 ? F_WRAP64 : F_WRAP32, s);
      chk(hop_right(d, f64, s));
    }
    // G = e^{-dtau K} T
    HopDesc d2{};
    d2.L = I.L; d2.mats = I.mats;
    d2.X = I.Tw; d2.sX = (long)NN(); d2.Y = Gcur(); d2.sY = (long)NN();
    d2.r = f64 ? (const void *)I.rm : (const void *)I.rtm;
    Timed tm(c, f64 ? F_WRAP64 : F_WRAP32, s);
    chk(hop_left(d2, f64, s));
  }

  // the same wrap as two batched MFMA GEMMs with the dense exponentials
  void wrap_gemm() {
    const bool f64 = I.cur64;
    const long bs = (long)NN();
    GemmDesc d = gemm_desc(I.N, I.mats);
    // T = (D G D^{-1}) e^{+dtau K}
    d.A = Gcur(); d.sA = bs; d.B = f64 ? (void *)I.Ep : (void *)I.Etp; d.sB = 0; d.C = I.Tw; d.sC = bs;
    const size_t esz = f64 ? 8 : 4;
    d.rs = I.dv; d.srs = 2L * I.N;
    d.ks = (char *)I.dv + esz * I.N; d.sks = 2L * I.N;
    {
      Timed tm(c, f64 ? F_WRAP64 : F_WRAP32, s);
      chk(f64 ? gemm_f64(d, false, false, s) : gemm_f32(d, false, false, s));
    }
    // G = e^{-dtau K} T
    GemmDesc d2 = gemm_desc(I.N, I.mats);
    d2.A = f64 ? (void *)I.Em : (void *)I.Etm; d2.sA = 0; d2.B = I.Tw; d2.sB = bs; d2.C = Gcur(); d2.sC = bs;
    Timed tm(c, f64 ? F_WRAP64 : F_WRAP32, s);
    chk(f64 ? gemm_f64(d2, false, false, s) : gemm_f32(d2, false, false, s));
  }

  void stabilise(int l) {
    wait_left();
    const int b = (l - 1) / I.n_stab;
    block_product(b);
    right_update(b);
    fresh(b, false, I.Gf);
    replace(l == I.Lam ? 1 : l + 1, b == 0 ? 2 : 1, c->opt.drift_abort);
  }

  void slice(int l) {
    if (l == 1) begin_sweep();
    flip(l);
    wrap();
    if (l % I.n_stab == 0 || l == I.Lam) stabilise(l);
  }

  // The left factors of a sweep are rebuilt from the block products of the
  // sweep before it.  That rebuild runs on the aux stream at the start of the
  // sweep, under the slices of the first block, which touch neither the
  // block products nor the QR scratch; the first recomputation waits for it.
  void begin_sweep() {
    if (!I.left_stale) return;
    chk(hipEventRecord(I.ev_main, I.s));
    chk(hipStreamWaitEvent(I.aux, I.ev_main, 0));
    s = I.aux;
    left_rebuild();
    s = I.s;
    chk(hipEventRecord(I.ev_left, I.aux));
    I.left_pending = true;
    I.left_stale = false;
  }

  // sweep counter; the left factors are now due for a rebuild
  void end_of_sweep() {
    chk(bump_counter(I.sweep_ctr, I.s));
    I.left_stale = true;
  }

  // measurement of the sweep just finished: Gf holds G(0) = G(1) fresh, the
  // right chain after each block is current, the left factors are rebuilt
  // here if the next sweep has not done so.
  void measure() {
    wait_left();
    if (I.left_stale) {
      left_rebuild();
      I.left_stale = false;
    }
    chk(meas_begin(I.ms, I.C, s));
    chk(meas_docc(I.ms, I.Gf, I.C, I.N, s));
    chk(meas_sc(I.ms, I.Gf, I.C, I.L, s));
    chk(hipMemcpyAsync(I.Gt, I.Gf, sizeof(double) * I.mats * NN(), hipMemcpyDeviceToDevice, s));
    chk(meas_gk(I.ms, I.Gt, I.C, I.L, 0, s));
    for (int l = 1; l <= I.Lam; ++l) {
      if (l % I.n_stab == 0 || l == I.Lam) {
        fresh((l - 1) / I.n_stab, true, I.Gt);      // stable G(tau_l, 0) at a block boundary
      } else {
        // G(tau_l, 0) = B_l G(tau_{l-1}, 0) = e^{-dtau K} diag(d_l) G(tau_{l-1}, 0)
        chk(slice_scales(I.h, I.C, I.Lam, I.N, l, l, std::exp(I.lambda), std::exp(-I.lambda), I.dvD, s));
        hop64(I.Gt, I.Pw, I.dvD, I.N);
        chk(hipMemcpyAsync(I.Gt, I.Pw, sizeof(double) * I.mats * NN(), hipMemcpyDeviceToDevice, s));
      }
      chk(meas_gk(I.ms, I.Gt, I.C, I.L, l, s));
    }
    chk(meas_end(I.ms, I.C, s));
  }
};

// every shard's main stream starts after the work already on the context stream
hipError_t fork(bss_ctx *c) {
  hipError_t e = hipEventRecord(c->ev_fork, c->stream);
  for (auto &I : c->sh)
    if (e == hipSuccess) e = hipStreamWaitEvent(I.s, c->ev_fork, 0);
  return e;
}

// the context stream waits for all work of every shard (main and aux)
hipError_t join(bss_ctx *c) {
  hipError_t e = hipSuccess;
  for (auto &I : c->sh) {
    if (e == hipSuccess) e = hipEventRecord(I.ev_main, I.s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, I.ev_main, 0);
    if (e == hipSuccess && I.left_pending) e = hipStreamWaitEvent(c->stream, I.ev_left, 0);
  }
  return e;
}

bss_status check_err(bss_ctx *c) {
  if (c->poisoned) return fail(c, BSS_E_STATE, "context poisoned by an earlier numerical failure");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) { c->poisoned = true; return fail(c, BSS_E_DEVICE, std::string("device error: ") + hipGetErrorString(e)); }
  int herr = 0;
  e = hipMemcpy(&herr, c->err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) { c->poisoned = true; return fail(c, BSS_E_DEVICE, hipGetErrorString(e)); }
  if (herr & 8) { c->poisoned = true; return fail(c, BSS_E_STATE, "sweep ran past the supplied accept history"); }
  if (herr) {
    c->poisoned = true;
    std::string m = "numerical failure:";
    if (herr & 16) m += " non-finite determinant ratio;";
    if (herr & 32) m += " non-positive determinant ratio;";
    if (herr & 2) m += " wrap drift above drift_abort;";
    if (herr & 4) m += " non-finite recomputed Green function;";
    return fail(c, BSS_E_NUMERICAL, m);
  }
  return BSS_OK;
}

bss_status usable(bss_ctx *c) {
  if (!c) return BSS_E_INVALID_ARG;
  if (c->poisoned) return fail(c, BSS_E_STATE, "context poisoned by an earlier failure");
  return BSS_OK;
}

bss_status exec_failed(bss_ctx *c, const Exec &x) {
  c->poisoned = true;
  return fail(c, BSS_E_DEVICE, hipGetErrorString(x.e));
}

bss_status create_impl(const bss_instance *in, int n, const bss_options *opt_in, bss_ctx **out) {
  if (!out) return BSS_E_INVALID_ARG;
  *out = nullptr;
  if (!in || n < 1) return BSS_E_INVALID_ARG;
  std::string why;
  if (!check_options(opt_in, why)) return BSS_E_INVALID_ARG;
  bss_options opt;
  bss_options_default(&opt);
  if (opt_in) opt = *opt_in;
  std::vector<Shard> v;
  std::vector<UInst> u;
  bss_status code;
  if (!resolve(in, n, opt, v, u, why, code)) return code;
  bss_ctx *c = new (std::nothrow) bss_ctx;
  if (!c) return BSS_E_OUT_OF_MEMORY;
  c->opt = opt;
  c->fp64 = opt.precision == BSS_PREC_FP64;
  c->sh = v;
  c->ui = u;
  c->fam.resize(F_COUNT);
  for (int f = 0; f < F_COUNT; ++f) c->fam[f].name = FAM_NAMES[f];
  auto bail = [&](bss_status s) { bss_destroy(c); return s; };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(BSS_E_DEVICE);
  if (opt.stream) c->stream = (hipStream_t)opt.stream;
  else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return bail(BSS_E_DEVICE);
    c->own_stream = true;
  }
  if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) return bail(BSS_E_DEVICE);
  for (auto &I : c->sh) {
    if (hipStreamCreateWithFlags(&I.s, hipStreamNonBlocking) != hipSuccess) return bail(BSS_E_DEVICE);
    if (hipStreamCreateWithFlags(&I.aux, hipStreamNonBlocking) != hipSuccess) return bail(BSS_E_DEVICE);
    if (hipEventCreateWithFlags(&I.ev_main, hipEventDisableTiming) != hipSuccess) return bail(BSS_E_DEVICE);
    if (hipEventCreateWithFlags(&I.ev_left, hipEventDisableTiming) != hipSuccess) return bail(BSS_E_DEVICE);
  }
  const size_t need = total_bytes(c->sh, c->ui, opt) + 4096;
  if (opt.workspace) {
    if (opt.workspace_bytes < need) return bail(BSS_E_OUT_OF_MEMORY);
    c->mem = (char *)opt.workspace;
    c->mem_bytes = opt.workspace_bytes;
  } else {
    if (hipMalloc(&c->mem, need) != hipSuccess) { c->mem = nullptr; return bail(BSS_E_OUT_OF_MEMORY); }
    c->own_mem = true;
    c->mem_bytes = need;
  }
  Carver cv;
  cv.base = c->mem;
  layout_all(c->sh, c->ui, opt, cv, &c->err);
  c->profile = (opt.flags & BSS_FLAG_PROFILE) != 0;   // creation work is dropped from the profile below
  c->graphs = !c->profile && !(opt.flags & BSS_FLAG_NO_GRAPH);
  hipStream_t s = c->stream;
  if (hipMemsetAsync(c->mem, 0, cv.off, s) != hipSuccess) return bail(BSS_E_DEVICE);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(BSS_E_DEVICE);
  for (auto &I : c->sh) {
    std::vector<int64_t> ones(I.C, 1);
    if (hipMemcpy(I.ms.binsize, ones.data(), sizeof(int64_t) * I.C, hipMemcpyHostToDevice) != hipSuccess)
      return bail(BSS_E_DEVICE);
  }
  if (fork(c) != hipSuccess) return bail(BSS_E_DEVICE);
  for (auto &I : c->sh) {
    Exec x(c, I);
    x.chk(build_exp(I.L, I.t, I.dtau, I.Em, I.Ep, I.Etm, I.Etp, I.rm, I.rp, I.rtm, I.rtp, I.s));
    x.initialise(true);
    if (x.e != hipSuccess) { c->last_error = hipGetErrorString(x.e); return bail(BSS_E_DEVICE); }
  }
  if (join(c) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return bail(BSS_E_DEVICE);
  for (auto &f : c->fam) {
    for (auto &p : f.pending) { c->pool.push_back(p.first); c->pool.push_back(p.second); }
    f.pending.clear();
  }
  *out = c;
  return BSS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void bss_options_default(bss_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(bss_options);
  o->precision = BSS_PREC_FP64;
  o->drift_abort = 0.1;
}

bss_status bss_create(int32_t L, double U, double t, double beta, double dtau, uint64_t seed, int32_t n_chains,
                      const bss_options *opt, bss_ctx **out) {
  bss_instance in{L, U, t, beta, dtau, seed, n_chains};
  return create_impl(&in, 1, opt, out);
}

bss_status bss_create_batch(const bss_instance *inst, int32_t n_inst, const bss_options *opt, bss_ctx **out) {
  return create_impl(inst, n_inst, opt, out);
}

bss_status bss_workspace_size(const bss_instance *inst, int32_t n_inst, const bss_options *opt_in, size_t *bytes) {
  if (!inst || n_inst < 1 || !bytes) return BSS_E_INVALID_ARG;
  std::string why;
  if (!check_options(opt_in, why)) return BSS_E_INVALID_ARG;
  bss_options opt;
  bss_options_default(&opt);
  if (opt_in) opt = *opt_in;
  std::vector<Shard> v;
  std::vector<UInst> u;
  bss_status code;
  if (!resolve(inst, n_inst, opt, v, u, why, code)) return code;
  *bytes = total_bytes(v, u, opt) + 4096 + 256;
  return BSS_OK;
}

}  // extern "C"

namespace {

// Enqueue n whole sweeps (every shard at slice 1) between a fork from and a
// join into the context stream.  The host-side state it leaves (slice 1, the
// precision of slice 1, a pending left rebuild) is the same after every
// sweep, which is what lets one captured sweep stand for any of them.
bss_status enqueue_sweeps(bss_ctx *c, int n_sweeps, bool measure) {
  HIP_TRY(c, fork(c));
  int lam_max = 0;
  for (auto &I : c->sh) lam_max = std::max(lam_max, I.Lam);
  std::vector<Exec> xs;
  xs.reserve(c->sh.size());
  for (auto &I : c->sh) xs.emplace_back(c, I);
  for (int sw = 0; sw < n_sweeps; ++sw) {
    // slice by slice across the shards, so that their streams overlap
    for (int l = 1; l <= lam_max; ++l)
      for (auto &x : xs) {
        if (l > x.I.Lam) continue;
        x.slice(l);
        if (l == x.I.Lam) x.end_of_sweep();
      }
    if (measure)
      for (auto &x : xs) x.measure();
    for (auto &x : xs)
      if (x.e != hipSuccess) return exec_failed(c, x);
  }
  HIP_TRY(c, join(c));
  return BSS_OK;
}

// Enqueue slices [l_from, l_to] of one sweep for every shard (l_from = 1
// starts the sweep: the left rebuild is launched first, on the aux streams),
// between a fork from and a join into the context stream.
bss_status enqueue_range(bss_ctx *c, int l_from, int l_to) {
  HIP_TRY(c, fork(c));
  std::vector<Exec> xs;
  xs.reserve(c->sh.size());
  for (auto &I : c->sh) xs.emplace_back(c, I);
  if (l_from == 1)
    for (auto &x : xs) x.begin_sweep();
  for (int l = l_from; l <= l_to; ++l)
    for (auto &x : xs) {
      if (l > x.I.Lam) continue;
      x.slice(l);
      if (l == x.I.Lam) x.end_of_sweep();
    }
  for (auto &x : xs)
    if (x.e != hipSuccess) return exec_failed(c, x);
  HIP_TRY(c, join(c));
  return BSS_OK;
}

bool capture_range(bss_ctx *c, int l_from, int l_to, hipGraphExec_t *out) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const bss_status st = enqueue_range(c, l_from, l_to);
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    ok = st == BSS_OK && e == hipSuccess && g != nullptr;
  }
  hipGraphExec_t ex = nullptr;
  if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok && ex) {
    (void)hipGraphExecDestroy(ex);
    ex = nullptr;
  }
  *out = ex;
  return ok;
}

// Capture one unmeasured sweep into two executable graphs, both starting
// from and ending on the context stream: the first holds the left rebuild of
// the sweep before (aux streams) beside the slices up to the first
// recomputation, the second the rest of the sweep.  Every cross-stream
// dependency inside a capture is thus a fork from a stream already in it, or
// a join into the context stream; a shard stream never waits on its aux
// stream inside a capture.  Two captures with such a wait (the measured
// sweep, and the rebuild joined into the first recomputation) each crashed
// the host process inside the HIP runtime, and the cause could not be shown,
// so that form is not captured.  Measured sweeps always launch directly.
// Returns false if the runtime refuses a capture; the caller then stays with
// direct launches.
void release_graph(bss_ctx::SweepGraph &sg) {
  for (auto &g : sg.g)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  if (sg.ev_fork) { (void)hipEventDestroy(sg.ev_fork); sg.ev_fork = nullptr; }
  for (auto &e : sg.ev)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
}

bool capture_sweep(bss_ctx *c, bss_ctx::SweepGraph &sg) {
  const size_t n = c->sh.size();
  // the capture's own events
  bool ok = hipEventCreateWithFlags(&sg.ev_fork, hipEventDisableTiming) == hipSuccess;
  sg.ev.assign(2 * n, nullptr);
  for (auto &e : sg.ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) { release_graph(sg); return false; }
  hipEvent_t keep_fork = c->ev_fork;
  std::vector<hipEvent_t> keep(2 * n);
  std::vector<bool> pend(n), cur(n), stale(n);
  int l_first = 1 << 30, lam_max = 0;
  c->ev_fork = sg.ev_fork;
  for (size_t i = 0; i < n; ++i) {
    Shard &I = c->sh[i];
    keep[2 * i] = I.ev_main;
    keep[2 * i + 1] = I.ev_left;
    I.ev_main = sg.ev[2 * i];
    I.ev_left = sg.ev[2 * i + 1];
    pend[i] = I.left_pending;
    cur[i] = I.cur64;
    stale[i] = I.left_stale;
    I.left_pending = false;
    I.left_stale = true;   // every replay starts with the rebuild of the sweep before
    l_first = std::min(l_first, std::min(I.n_stab, I.Lam));
    lam_max = std::max(lam_max, I.Lam);
  }
  ok = capture_range(c, 1, l_first - 1, &sg.g[0]);
  // the first part's join has ordered the context stream after the rebuilds
  for (auto &I : c->sh) I.left_pending = false;
  if (ok) ok = capture_range(c, l_first, lam_max, &sg.g[1]);
  // a capture enqueues nothing: restore the host-side state it advanced and
  // the events of direct launches
  c->ev_fork = keep_fork;
  for (size_t i = 0; i < n; ++i) {
    Shard &I = c->sh[i];
    I.ev_main = keep[2 * i];
    I.ev_left = keep[2 * i + 1];
    I.left_pending = pend[i];
    I.cur64 = cur[i];
    I.left_stale = stale[i];
  }
  c->poisoned = false;
  (void)hipGetLastError();
  if (!ok) release_graph(sg);
  return ok;
}

std::vector<int> fp32_key(const bss_ctx *c) {
  std::vector<int> k;
  for (auto &I : c->sh) k.push_back(I.m32);
  return k;
}

// (the caller has synchronised the context stream the graphs run on)
void destroy_graphs(bss_ctx *c) {
  for (auto &sg : c->gcache) release_graph(sg);
  c->gcache.clear();
}

// the captured sweep of the current FP32 slice counts (captured on first
// use; at most 8 kept); nullptr if the runtime refuses the capture, after
// which the context launches directly
const bss_ctx::SweepGraph *sweep_graph(bss_ctx *c) {
  const std::vector<int> key = fp32_key(c);
  for (auto &sg : c->gcache)
    if (sg.key == key) return &sg;
  if (c->gcache.size() >= 8) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) { c->graphs = false; return nullptr; }
    release_graph(c->gcache.front());
    c->gcache.erase(c->gcache.begin());
  }
  bss_ctx::SweepGraph sg;
  sg.key = key;
  if (!capture_sweep(c, sg)) {
    c->graphs = false;
    return nullptr;
  }
  c->gcache.push_back(sg);
  return &c->gcache.back();
}

int64_t x_negs(const std::vector<ChainStats> &cs) {
  int64_t n = 0;
  for (auto &x : cs) n += x.negs;
  return n;
}

int fp32_count(const Shard &I) {
  int n = 0;
  for (int l = 1; l <= I.Lam; ++l) n += fp32_slice(I, l) ? 1 : 0;
  return n;
}

// Drift controller of mixed precision with the automatic FP32 slice count.
// After a sweep, the largest relative wrap drift d of each adapting
// instance's chains in that sweep moves the next sweep's count by one: down
// if d > target / 2; up (to at most the automatic count) if d e^{2 lambda}
// < target / 2, e^{2 lambda} being the growth one more FP32 slice brings
// (the spread of a slice's diagonal factors amplifies an earlier rounding
// error once per wrap).  G is then converted to the precision slice 1 needs.
// With fp32_adapt_sweeps = n > 0 an instance stops adapting after the n-th
// adjusted sweep and holds its count from then on ("settled"): its sweeps can
// then be captured like those of a fixed count, and it keeps the FP32 guard
// (settled_fuse applies the fuse to it).
bss_status adapt_fp32(bss_ctx *c) {
  bool any = false;
  for (auto &I : c->sh) any = any || I.adapt;
  if (!any) return BSS_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const double target = c->opt.fp32_drift_target > 0.0 ? c->opt.fp32_drift_target : 1e-3;
  bool changed = false;
  std::vector<int> next(c->sh.size());
  for (size_t k = 0; k < c->sh.size(); ++k) {
    Shard &I = c->sh[k];
    next[k] = I.m32;
    if (!I.adapt) continue;
    std::vector<ChainStats> cs(I.C);
    HIP_TRY(c, hipMemcpy(cs.data(), I.stats, sizeof(ChainStats) * I.C, hipMemcpyDeviceToHost));
    double d = 0.0;
    int64_t rej = 0;
    for (auto &x : cs) {
      d = std::isnan(x.rdrift_sweep) ? INFINITY : std::max(d, x.rdrift_sweep);
      rej += x.fp32_rejected;
    }
    if (rej > I.fp32_rej_seen) {   // the fuse: FP32 is not safe for this instance
      I.fp32_rej_seen = rej;
      I.adapt = false;
      I.fused = true;
      next[k] = 0;
      changed = changed || I.m32 != 0;
      continue;
    }
    if (d > 0.5 * target) next[k] = std::max(0, I.m32 - 1);
    else if (d * std::exp(2.0 * I.lambda) < 0.5 * target) next[k] = std::min(I.m32_max, I.m32 + 1);
    changed = changed || next[k] != I.m32;
    I.adapted += 1;
    if (c->opt.fp32_adapt_sweeps > 0 && I.adapted >= c->opt.fp32_adapt_sweeps) {
      I.adapt = false;
      I.settled = true;
    }
  }
  if (!changed) return BSS_OK;
  HIP_TRY(c, fork(c));
  for (size_t k = 0; k < c->sh.size(); ++k) {
    Shard &I = c->sh[k];
    if (next[k] == I.m32) continue;
    I.m32 = next[k];
    Exec x(c, I);
    x.use_precision(1);
    if (x.e != hipSuccess) return exec_failed(c, x);
  }
  HIP_TRY(c, join(c));
  return BSS_OK;
}

// The fuse of settled instances: a ratio rejected in their FP32 slices since
// the last look switches the instance to FP64, as the controller does after a
// sweep.  Their sweeps may have been replayed from a captured graph of the
// held counts; after a fuse the context launches directly, so that no second
// set of counts is ever captured in it (see bss_sweep).  Runs at the start of
// bss_sweep; waits for the work already issued.
bss_status settled_fuse(bss_ctx *c) {
  bool any = false;
  for (auto &I : c->sh) any = any || (I.settled && I.m32 > 0);
  if (!any) return BSS_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<size_t> hit;
  for (size_t k = 0; k < c->sh.size(); ++k) {
    Shard &I = c->sh[k];
    if (!I.settled || I.m32 == 0) continue;
    std::vector<ChainStats> cs(I.C);
    HIP_TRY(c, hipMemcpy(cs.data(), I.stats, sizeof(ChainStats) * I.C, hipMemcpyDeviceToHost));
    int64_t rej = 0;
    for (auto &x : cs) rej += x.fp32_rejected;
    if (rej > I.fp32_rej_seen) {
      I.fp32_rej_seen = rej;
      I.settled = false;
      I.fused = true;
      hit.push_back(k);
    }
  }
  if (hit.empty()) return BSS_OK;
  c->graphs = false;
  HIP_TRY(c, fork(c));
  for (size_t k : hit) {
    Shard &I = c->sh[k];
    I.m32 = 0;
    Exec x(c, I);
    x.use_precision(1);
    if (x.e != hipSuccess) return exec_failed(c, x);
  }
  HIP_TRY(c, join(c));
  return BSS_OK;
}

}  // namespace

extern "C" {

bss_status bss_sweep(bss_ctx *c, int32_t n_sweeps, int32_t measure) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (n_sweeps < 0) return fail(c, BSS_E_INVALID_ARG, "n_sweeps must be >= 0");
  for (auto &I : c->sh)
    if (I.slice != 1) return fail(c, BSS_E_STATE, "an instance is part-way through a sweep");
  if ((st = settled_fuse(c)) != BSS_OK) return st;
  for (int done = 0; done < n_sweeps;) {
    // while the drift controller adapts, the FP32 slice counts may change
    // after every sweep, so sweeps are issued one at a time, and launched
    // directly: a process that had swept a controlled context through
    // captured sweeps of several counts crashed in the HIP runtime when it
    // went on to the next context (twice at the same point, cause not found),
    // so a context captures sweeps only while its slice precisions no longer
    // change (fixed counts, or counts held once settled) and at most one set
    // of counts (a fuse after settling turns capture off)
    bool adapt = false;
    for (auto &I : c->sh) adapt = adapt || I.adapt;
    const int n = adapt ? 1 : n_sweeps - done;
    const bss_ctx::SweepGraph *sg = (c->graphs && !measure && !adapt) ? sweep_graph(c) : nullptr;
    if (sg) {
      for (int sw = 0; sw < n; ++sw) {
        HIP_TRY(c, hipGraphLaunch(sg->g[0], c->stream));
        HIP_TRY(c, hipGraphLaunch(sg->g[1], c->stream));
      }
      // the replays leave what direct launches would: slice 1 in its
      // precision, every left rebuild waited for on the context stream
      for (auto &I : c->sh) {
        I.cur64 = !fp32_slice(I, 1);
        I.left_pending = false;
        I.left_stale = true;
      }
    } else if ((st = enqueue_sweeps(c, n, measure != 0)) != BSS_OK) {
      return st;
    }
    for (auto &I : c->sh) {
      I.sweeps += n;
      I.slices_run += (int64_t)n * I.Lam;
      I.fp32_run += (int64_t)n * fp32_count(I);
    }
    done += n;
    if (adapt && (st = adapt_fp32(c)) != BSS_OK) return st;
  }
  return BSS_OK;
}

bss_status bss_step_slices(bss_ctx *c, int32_t n_slices) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (n_slices < 0) return fail(c, BSS_E_INVALID_ARG, "n_slices must be >= 0");
  if (n_slices == 0) return BSS_OK;
  HIP_TRY(c, fork(c));
  std::vector<Exec> xs;
  xs.reserve(c->sh.size());
  for (auto &I : c->sh) xs.emplace_back(c, I);
  for (int n = 0; n < n_slices; ++n)
    for (auto &x : xs) {
      Shard &I = x.I;
      I.slices_run += 1;
      I.fp32_run += fp32_slice(I, I.slice) ? 1 : 0;
      x.slice(I.slice);
      if (I.slice == I.Lam) {
        x.end_of_sweep();
        I.slice = 1;
        I.sweeps += 1;
      } else {
        I.slice += 1;
      }
      if (x.e != hipSuccess) return exec_failed(c, x);
    }
  HIP_TRY(c, join(c));
  return BSS_OK;
}

}  // extern "C"

namespace {

bss_status pick(bss_ctx *c, int32_t inst, UInst **U) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (inst < 0 || inst >= (int)c->ui.size()) return fail(c, BSS_E_INVALID_ARG, "instance index out of range");
  *U = &c->ui[inst];
  return BSS_OK;
}

// the shard of an instance that holds chain `chain`
Shard &shard_of(bss_ctx *c, const UInst &U, int chain) {
  for (int k = 0; k + 1 < U.count; ++k) {
    Shard &I = c->sh[U.first + k];
    if (chain < I.chain0 + I.C) return I;
  }
  return c->sh[U.first + U.count - 1];
}

}  // namespace

extern "C" {

bss_status bss_get_green(bss_ctx *c, int32_t inst, int32_t chain, int32_t spin, double *out) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (chain < 0 || chain >= U->C || (spin != 0 && spin != 1) || !out) return fail(c, BSS_E_INVALID_ARG, "bad chain/spin/out");
  if ((st = check_err(c)) != BSS_OK) return st;
  Shard &I = shard_of(c, *U, chain);
  const size_t n = nn(I);
  const size_t off = (size_t)(2 * (chain - I.chain0) + spin) * n;
  if (I.cur64) {
    HIP_TRY(c, hipMemcpy(out, I.G64 + off, sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(n);
    HIP_TRY(c, hipMemcpy(tmp.data(), I.G32 + off, sizeof(float) * n, hipMemcpyDeviceToHost));
    for (size_t e = 0; e < n; ++e) out[e] = tmp[e];
  }
  return BSS_OK;
}

bss_status bss_debug_set_green(bss_ctx *c, int32_t inst, int32_t chain, int32_t spin, int32_t i, int32_t j,
                               double value) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (chain < 0 || chain >= U->C || (spin != 0 && spin != 1) || i < 0 || i >= U->N || j < 0 || j >= U->N)
    return fail(c, BSS_E_INVALID_ARG, "bad chain/spin/indices");
  if ((st = check_err(c)) != BSS_OK) return st;
  Shard &I = shard_of(c, *U, chain);
  const size_t off = (size_t)(2 * (chain - I.chain0) + spin) * nn(I) + (size_t)i * I.N + j;
  if (I.cur64) {
    HIP_TRY(c, hipMemcpy(I.G64 + off, &value, sizeof(double), hipMemcpyHostToDevice));
  } else {
    const float v = (float)value;
    HIP_TRY(c, hipMemcpy(I.G32 + off, &v, sizeof(float), hipMemcpyHostToDevice));
  }
  return BSS_OK;
}

bss_status bss_get_field(bss_ctx *c, int32_t inst, int32_t chain, int8_t *out) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (chain < 0 || chain >= U->C || !out) return fail(c, BSS_E_INVALID_ARG, "bad chain/out");
  if ((st = check_err(c)) != BSS_OK) return st;
  Shard &I = shard_of(c, *U, chain);
  const size_t n = (size_t)I.Lam * I.N;
  HIP_TRY(c, hipMemcpy(out, I.h + (size_t)(chain - I.chain0) * n, n, hipMemcpyDeviceToHost));
  return BSS_OK;
}

bss_status bss_set_field(bss_ctx *c, int32_t inst, int32_t chain, const int8_t *in) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (chain < 0 || chain >= U->C || !in) return fail(c, BSS_E_INVALID_ARG, "bad chain/in");
  for (auto &J : c->sh)
    if (J.slice != 1) return fail(c, BSS_E_STATE, "set_field needs every instance at slice 1");
  Shard &I = shard_of(c, *U, chain);
  const size_t n = (size_t)I.Lam * I.N;
  for (size_t e = 0; e < n; ++e)
    if (in[e] != 1 && in[e] != -1) return fail(c, BSS_E_INVALID_ARG, "field entries must be +-1");
  if ((st = check_err(c)) != BSS_OK) return st;
  HIP_TRY(c, hipMemcpy(I.h + (size_t)(chain - I.chain0) * n, in, n, hipMemcpyHostToDevice));
  HIP_TRY(c, fork(c));
  Exec x(c, I);
  x.initialise(false);
  if (x.e != hipSuccess) return exec_failed(c, x);
  HIP_TRY(c, join(c));
  return check_err(c);
}

bss_status bss_set_trace(bss_ctx *c, int32_t inst, const uint8_t *accept, int32_t n_sweeps) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (!(c->opt.flags & BSS_FLAG_REPLAY_TRACE)) return fail(c, BSS_E_STATE, "context not created with BSS_FLAG_REPLAY_TRACE");
  if (!accept || n_sweeps < 1 || n_sweeps > U->trace_alloc) return fail(c, BSS_E_INVALID_ARG, "n_sweeps must be in 1..trace_sweeps");
  for (int k = 0; k < U->count; ++k)
    if (c->sh[U->first + k].slice != 1) return fail(c, BSS_E_STATE, "set_trace needs the instance at slice 1");
  if ((st = check_err(c)) != BSS_OK) return st;
  const size_t n = (size_t)n_sweeps * U->C * U->Lam * U->N;
  HIP_TRY(c, hipMemcpy(U->trace, accept, n, hipMemcpyHostToDevice));
  int64_t base = c->sh[U->first].sweeps;
  HIP_TRY(c, hipMemcpy(U->trace_base, &base, sizeof(base), hipMemcpyHostToDevice));
  U->trace_cap = n_sweeps;   // sweeping past this window is an error
  // the flip launches carry the window length: captured sweeps are stale
  destroy_graphs(c);
  return BSS_OK;
}

bss_status bss_get_trace(bss_ctx *c, int32_t inst, uint8_t *accept, int32_t n_sweeps) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (!(c->opt.flags & BSS_FLAG_RECORD_TRACE)) return fail(c, BSS_E_STATE, "context not created with BSS_FLAG_RECORD_TRACE");
  if (!accept || n_sweeps < 1 || n_sweeps > U->trace_cap) return fail(c, BSS_E_INVALID_ARG, "n_sweeps must be in 1..trace_sweeps");
  if ((st = check_err(c)) != BSS_OK) return st;
  const size_t n = (size_t)n_sweeps * U->C * U->Lam * U->N;
  HIP_TRY(c, hipMemcpy(accept, U->trace, n, hipMemcpyDeviceToHost));
  return BSS_OK;
}

bss_status bss_get_stats(bss_ctx *c, int32_t inst, bss_stats *out) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (!out) return fail(c, BSS_E_INVALID_ARG, "out is NULL");
  if ((st = check_err(c)) != BSS_OK) return st;
  std::memset(out, 0, sizeof(*out));
  out->sign = 1;
  double dsum = 0, rsum = 0;
  int64_t dcnt = 0, run = 0, run32 = 0, negs = 0;
  bool settled = true;
  for (int k = 0; k < U->count; ++k) {
    const Shard &I = c->sh[U->first + k];
    std::vector<ChainStats> cs(I.C);
    HIP_TRY(c, hipMemcpy(cs.data(), I.stats, sizeof(ChainStats) * I.C, hipMemcpyDeviceToHost));
    for (auto &x : cs) {
      out->proposals += x.proposals;
      out->accepted += x.accepted;
      out->logw += x.logw;
      out->drift_max = std::max(out->drift_max, x.drift_max);
      out->drift_rel_max = std::max(out->drift_rel_max, x.rdrift_max);
      dsum += x.drift_sum;
      rsum += x.rdrift_sum;
      dcnt += x.drift_count;
    }
    out->sweeps = I.sweeps;
    out->N = I.N; out->Lambda = I.Lam; out->delay_k = I.k; out->n_stab = I.n_stab;
    out->fp32_slices = I.m32;
    run += I.slices_run;
    run32 += I.fp32_run;
    negs += x_negs(cs);
    for (auto &x : cs) out->fp32_rejected += x.fp32_rejected;
    out->fp32_fused = out->fp32_fused || I.fused;
    settled = settled && I.settled;
  }
  out->fp32_settled = settled ? 1 : 0;
  out->sign = (negs % 2) ? -1 : 1;
  out->fp32_fraction = run ? (double)run32 / (double)run : 0.0;
  out->drift_mean = dcnt ? dsum / dcnt : 0.0;
  out->drift_rel_mean = dcnt ? rsum / dcnt : 0.0;
  out->sweep_graph = c->gcache.empty() ? 0 : 1;
  out->n_chains = U->C;
  out->shards = U->count;
  return BSS_OK;
}

}  // extern "C"

namespace {

// per-chain measurement arrays of one instance, in chain order
// per-chain bins of one observable of an instance, in chain order: the double
// occupancy ([C][NBINS]), G(tau, k) or C(r) ([C][nbins_g][len])
enum Obs { OBS_DOCC, OBS_GK, OBS_SC };

bss_status fetch_meas(bss_ctx *c, const UInst &U, Obs which, std::vector<double> &docc, std::vector<double> &gk,
                      std::vector<int64_t> &count, std::vector<int64_t> &binsize, size_t &glen) {
  const Shard &F = c->sh[U.first];
  glen = (size_t)(which == OBS_SC ? F.ms.sclen : F.ms.glen);
  const size_t gper = (size_t)F.ms.nbins_g * glen;
  docc.resize((size_t)U.C * NBINS);
  gk.resize(which == OBS_DOCC ? 0 : (size_t)U.C * gper);
  count.resize(U.C);
  binsize.resize(U.C);
  for (int k = 0; k < U.count; ++k) {
    const Shard &I = c->sh[U.first + k];
    const size_t c0 = I.chain0;
    HIP_TRY(c, hipMemcpy(docc.data() + c0 * NBINS, I.ms.docc, sizeof(double) * I.C * NBINS, hipMemcpyDeviceToHost));
    if (which != OBS_DOCC)
      HIP_TRY(c, hipMemcpy(gk.data() + c0 * gper, which == OBS_SC ? I.ms.sc : I.ms.gk, sizeof(double) * I.C * gper,
                           hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(count.data() + c0, I.ms.count, sizeof(int64_t) * I.C, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(binsize.data() + c0, I.ms.binsize, sizeof(int64_t) * I.C, hipMemcpyDeviceToHost));
  }
  return BSS_OK;
}

// mean and standard error of per-sample sums: samples[s] sums weights[s]
// measurements; the mean is over all measurements, the error is that of the
// mean of the per-sample means
void mean_err(const std::vector<std::vector<double>> &samples, const std::vector<double> &weights, size_t len,
              double *mean, double *err) {
  const size_t S = samples.size();
  double wsum = 0;
  for (double w : weights) wsum += w;
  for (size_t e = 0; e < len; ++e) {
    double m = 0;
    for (size_t s = 0; s < S; ++s) m += samples[s][e];
    m /= wsum;
    if (mean) mean[e] = m;
    if (err) {
      double acc = 0, mm = 0;
      size_t n = 0;
      for (size_t s = 0; s < S; ++s) if (weights[s] > 0) { mm += samples[s][e] / weights[s]; ++n; }
      mm = n ? mm / n : 0;
      for (size_t s = 0; s < S; ++s) if (weights[s] > 0) { const double d = samples[s][e] / weights[s] - mm; acc += d * d; }
      err[e] = n > 1 ? std::sqrt(acc / (n - 1) / n) : 0.0;
    }
  }
}

bss_status measure_common(bss_ctx *c, int32_t inst, Obs which, double *mean, double *err, int64_t len) {
  UInst *U;
  bss_status st = pick(c, inst, &U);
  if (st != BSS_OK) return st;
  if (!mean) return fail(c, BSS_E_INVALID_ARG, "mean is NULL");
  if (which == OBS_GK && len != (int64_t)(U->Lam + 1) * U->N) return fail(c, BSS_E_INVALID_ARG, "len must be (Lambda+1)*N");
  if (which == OBS_SC && len != (int64_t)U->N) return fail(c, BSS_E_INVALID_ARG, "len must be N");
  if ((st = check_err(c)) != BSS_OK) return st;
  const bool gk_wanted = which != OBS_DOCC;
  std::vector<double> docc, gk;
  std::vector<int64_t> count, binsize;
  size_t glen = 0;
  if ((st = fetch_meas(c, *U, which, docc, gk, count, binsize, glen)) != BSS_OK) return st;
  if (count[0] == 0) return fail(c, BSS_E_STATE, "no measurements accumulated");
  std::vector<std::vector<double>> samples;
  std::vector<double> weights;
  if (U->C >= 2) {
    for (int ch = 0; ch < U->C; ++ch) {
      if (gk_wanted) samples.emplace_back(gk.begin() + (size_t)ch * glen, gk.begin() + (size_t)(ch + 1) * glen);
      else {
        double s = 0;
        for (int b = 0; b < NBINS; ++b) s += docc[(size_t)ch * NBINS + b];
        samples.push_back({s});
      }
      weights.push_back((double)count[ch]);
    }
    mean_err(samples, weights, gk_wanted ? glen : 1, mean, err);
    return BSS_OK;
  }
  // one chain: complete bins for the error, everything for the mean
  const int64_t n = count[0], bs = binsize[0];
  const int full = (int)(n / bs);
  const int used = (int)((n + bs - 1) / bs);
  std::vector<double> tot(gk_wanted ? glen : 1, 0.0);
  for (int b = 0; b < used; ++b) {
    if (gk_wanted) for (size_t e = 0; e < glen; ++e) tot[e] += gk[(size_t)b * glen + e];
    else tot[0] += docc[b];
  }
  for (size_t e = 0; e < tot.size(); ++e) mean[e] = tot[e] / (double)n;
  if (err) {
    for (int b = 0; b < full; ++b) {
      if (gk_wanted) samples.emplace_back(gk.begin() + (size_t)b * glen, gk.begin() + (size_t)(b + 1) * glen);
      else samples.push_back({docc[b]});
      weights.push_back((double)bs);
    }
    if (full >= 2) mean_err(samples, weights, tot.size(), nullptr, err);
    else for (size_t e = 0; e < tot.size(); ++e) err[e] = 0.0;
  }
  return BSS_OK;
}

// Checkpoint layout: magic, number of instances, then per instance C, Lam,
// N, sweeps (int64 each) followed by, for all chains in order, the fields,
// the chain statistics, the double-occupancy bins, the G(tau,k) bins, the
// measurement counts and the bin sizes.  The layout does not depend on how
// the chains are sharded.
const uint64_t CK_MAGIC = 0x32504B4353534221ull;

size_t inst_ck_bytes(const bss_ctx *c, const UInst &U) {
  const Shard &F = c->sh[U.first];
  return 32 + (size_t)U.C * U.Lam * U.N + sizeof(ChainStats) * U.C + sizeof(double) * U.C * NBINS +
         sizeof(double) * U.C * F.ms.nbins_g * (F.ms.glen + F.ms.sclen) + 2 * sizeof(int64_t) * U.C;
}

// one per-chain section of the checkpoint: `per(I)` bytes per chain at `dev(I)`
template <typename Dev>
bss_status ck_section(bss_ctx *c, const UInst &U, char *&p, size_t per, Dev dev, bool save) {
  for (int k = 0; k < U.count; ++k) {
    Shard &I = c->sh[U.first + k];
    const size_t n = per * I.C;
    if (save) HIP_TRY(c, hipMemcpy(p, dev(I), n, hipMemcpyDeviceToHost));
    else HIP_TRY(c, hipMemcpy(dev(I), p, n, hipMemcpyHostToDevice));
    p += n;
  }
  return BSS_OK;
}

bss_status ck_transfer(bss_ctx *c, const UInst &U, char *&p, bool save) {
  const Shard &F = c->sh[U.first];
  const size_t gper = sizeof(double) * F.ms.nbins_g * F.ms.glen;
  bss_status st;
  if ((st = ck_section(c, U, p, (size_t)U.Lam * U.N, [](Shard &I) { return (void *)I.h; }, save)) != BSS_OK) return st;
  if ((st = ck_section(c, U, p, sizeof(ChainStats), [](Shard &I) { return (void *)I.stats; }, save)) != BSS_OK) return st;
  if ((st = ck_section(c, U, p, sizeof(double) * NBINS, [](Shard &I) { return (void *)I.ms.docc; }, save)) != BSS_OK) return st;
  if ((st = ck_section(c, U, p, gper, [](Shard &I) { return (void *)I.ms.gk; }, save)) != BSS_OK) return st;
  const size_t sper = sizeof(double) * F.ms.nbins_g * F.ms.sclen;
  if ((st = ck_section(c, U, p, sper, [](Shard &I) { return (void *)I.ms.sc; }, save)) != BSS_OK) return st;
  if ((st = ck_section(c, U, p, sizeof(int64_t), [](Shard &I) { return (void *)I.ms.count; }, save)) != BSS_OK) return st;
  return ck_section(c, U, p, sizeof(int64_t), [](Shard &I) { return (void *)I.ms.binsize; }, save);
}

}  // namespace

extern "C" {

bss_status bss_measure_gtau_k(bss_ctx *c, int32_t inst, double *mean, double *err, int64_t len) {
  return measure_common(c, inst, OBS_GK, mean, err, len);
}

bss_status bss_measure_double_occ(bss_ctx *c, int32_t inst, double *mean, double *err) {
  return measure_common(c, inst, OBS_DOCC, mean, err, 1);
}

bss_status bss_measure_spin_corr(bss_ctx *c, int32_t inst, double *mean, double *err, int64_t len) {
  return measure_common(c, inst, OBS_SC, mean, err, len);
}

bss_status bss_reset_measurements(bss_ctx *c) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if ((st = check_err(c)) != BSS_OK) return st;
  for (auto &I : c->sh) {
    HIP_TRY(c, hipMemset(I.ms.docc, 0, sizeof(double) * I.C * NBINS));
    HIP_TRY(c, hipMemset(I.ms.gk, 0, sizeof(double) * I.C * I.ms.nbins_g * I.ms.glen));
    HIP_TRY(c, hipMemset(I.ms.sc, 0, sizeof(double) * I.C * I.ms.nbins_g * I.ms.sclen));
    HIP_TRY(c, hipMemset(I.ms.count, 0, sizeof(int64_t) * I.C));
    std::vector<int64_t> ones(I.C, 1);
    HIP_TRY(c, hipMemcpy(I.ms.binsize, ones.data(), sizeof(int64_t) * I.C, hipMemcpyHostToDevice));
  }
  HIP_TRY(c, hipDeviceSynchronize());
  return BSS_OK;
}

bss_status bss_synchronize(bss_ctx *c) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  return check_err(c);
}

bss_status bss_reset_stats(bss_ctx *c) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if ((st = check_err(c)) != BSS_OK) return st;
  for (auto &I : c->sh) {
    std::vector<ChainStats> zero(I.C);
    std::memset(zero.data(), 0, sizeof(ChainStats) * I.C);
    HIP_TRY(c, hipMemcpy(I.stats, zero.data(), sizeof(ChainStats) * I.C, hipMemcpyHostToDevice));
    I.slices_run = I.fp32_run = 0;
    I.fp32_rej_seen = 0;
  }
  return BSS_OK;
}

bss_status bss_save(bss_ctx *c, void *buf, size_t *bytes) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (!bytes) return fail(c, BSS_E_INVALID_ARG, "bytes is NULL");
  size_t need = 16;
  for (auto &U : c->ui) need += inst_ck_bytes(c, U);
  if (!buf) { *bytes = need; return BSS_OK; }
  if (*bytes < need) return fail(c, BSS_E_INVALID_ARG, "buffer too small");
  for (auto &I : c->sh)
    if (I.slice != 1) return fail(c, BSS_E_STATE, "save needs every instance at slice 1");
  if ((st = check_err(c)) != BSS_OK) return st;
  char *p = (char *)buf;
  const uint64_t hdr[2] = {CK_MAGIC, (uint64_t)c->ui.size()};
  std::memcpy(p, hdr, 16); p += 16;
  for (auto &U : c->ui) {
    const int64_t meta[4] = {U.C, U.Lam, U.N, c->sh[U.first].sweeps};
    std::memcpy(p, meta, 32); p += 32;
    if ((st = ck_transfer(c, U, p, true)) != BSS_OK) return st;
  }
  *bytes = (size_t)(p - (char *)buf);
  return BSS_OK;
}

bss_status bss_load(bss_ctx *c, const void *buf, size_t bytes) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (!buf || bytes < 16) return fail(c, BSS_E_INVALID_ARG, "bad checkpoint buffer");
  const char *p = (const char *)buf, *end = p + bytes;
  uint64_t hdr[2];
  std::memcpy(hdr, p, 16); p += 16;
  if (hdr[0] != CK_MAGIC || hdr[1] != c->ui.size()) return fail(c, BSS_E_INVALID_ARG, "checkpoint does not match this context");
  for (auto &I : c->sh)
    if (I.slice != 1) return fail(c, BSS_E_STATE, "load needs every instance at slice 1");
  if ((st = check_err(c)) != BSS_OK) return st;
  // validate the whole buffer before any state changes
  {
    const char *q = p;
    for (auto &U : c->ui) {
      if ((size_t)(end - q) < inst_ck_bytes(c, U)) return fail(c, BSS_E_INVALID_ARG, "truncated checkpoint");
      int64_t meta[4];
      std::memcpy(meta, q, 32);
      if (meta[0] != U.C || meta[1] != U.Lam || meta[2] != U.N || meta[3] < 0)
        return fail(c, BSS_E_INVALID_ARG, "checkpoint instance mismatch");
      const int8_t *hf = (const int8_t *)(q + 32);
      for (size_t e = 0; e < (size_t)U.C * U.Lam * U.N; ++e)
        if (hf[e] != 1 && hf[e] != -1) return fail(c, BSS_E_INVALID_ARG, "corrupt field in checkpoint");
      q += inst_ck_bytes(c, U);
    }
  }
  for (auto &U : c->ui) {
    int64_t meta[4];
    std::memcpy(meta, p, 32); p += 32;
    char *w = const_cast<char *>(p);
    if ((st = ck_transfer(c, U, w, false)) != BSS_OK) return st;
    p = w;
    for (int k = 0; k < U.count; ++k) {
      Shard &I = c->sh[U.first + k];
      I.sweeps = meta[3];
      I.slice = 1;
      HIP_TRY(c, hipMemcpy(I.sweep_ctr, &I.sweeps, sizeof(int64_t), hipMemcpyHostToDevice));
    }
  }
  HIP_TRY(c, fork(c));
  for (auto &I : c->sh) {
    Exec x(c, I);
    x.initialise(false);
    if (x.e != hipSuccess) return exec_failed(c, x);
  }
  HIP_TRY(c, join(c));
  return check_err(c);
}

bss_status bss_get_profile(bss_ctx *c, bss_kernel_time *out, int32_t cap, int32_t *n_out) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (!c->profile) return fail(c, BSS_E_STATE, "context not created with BSS_FLAG_PROFILE");
  if (cap < 0 || (cap > 0 && !out)) return fail(c, BSS_E_INVALID_ARG, "bad output buffer");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto &f : c->fam) {
    for (auto &p : f.pending) {
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
      f.ms += ms;
      f.launches += 1;
      c->pool.push_back(p.first);
      c->pool.push_back(p.second);
    }
    f.pending.clear();
  }
  int n = 0;
  for (auto &f : c->fam) {
    if (n < cap) {
      std::memset(&out[n], 0, sizeof(bss_kernel_time));
      std::snprintf(out[n].name, sizeof(out[n].name), "%s", f.name);
      out[n].launches = f.launches;
      out[n].total_ms = f.ms;
    }
    ++n;
  }
  if (n_out) *n_out = n;
  return BSS_OK;
}

bss_status bss_reset_profile(bss_ctx *c) {
  bss_status st = usable(c);
  if (st != BSS_OK) return st;
  if (!c->profile) return fail(c, BSS_E_STATE, "context not created with BSS_FLAG_PROFILE");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto &f : c->fam) {
    for (auto &p : f.pending) { c->pool.push_back(p.first); c->pool.push_back(p.second); }
    f.pending.clear();
    f.launches = 0;
    f.ms = 0.0;
  }
  return BSS_OK;
}

}  // extern "C"

namespace {

struct Trial {
  int k = 0, ns = 0, m32 = 0;
  double ms = 0.0, drift = 0.0;
  bool ok = false;     // ran and stayed within the bound
};

// one candidate: fresh context, fields from the checkpoint, one untimed sweep
// (it captures the graph), then trial sweeps timed with events
bss_status run_trial(const bss_instance &in0, bss_options o, const std::vector<char> &ck, int trials, double bound,
                     Trial &t) {
  bss_instance in = in0;
  in.delay_k = in.n_stab = 0;   // the options below decide
  o.delay_k = t.k;
  o.n_stab = t.ns;
  o.fp32_slices = t.m32;
  o.workspace = nullptr;
  o.workspace_bytes = 0;
  bss_ctx *c = nullptr;
  bss_status st = create_impl(&in, 1, &o, &c);
  if (st != BSS_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.0f;
  st = bss_load(c, ck.data(), ck.size());
  if (st == BSS_OK) st = bss_sweep(c, 1, 0);
  if (st == BSS_OK) st = bss_reset_stats(c);
  if (st == BSS_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = BSS_E_DEVICE;
  if (st == BSS_OK && hipEventRecord(e0, c->stream) != hipSuccess) st = BSS_E_DEVICE;
  if (st == BSS_OK) st = bss_sweep(c, trials, 0);
  if (st == BSS_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = BSS_E_DEVICE;
  bss_stats s{};
  if (st == BSS_OK) st = bss_get_stats(c, 0, &s);   // synchronises
  if (st == BSS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BSS_E_DEVICE;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  bss_destroy(c);
  t.m32 = s.fp32_slices;
  if (st == BSS_E_NUMERICAL || st == BSS_E_STATE) {   // the chain broke down: out of bound
    t.ok = false;
    t.drift = INFINITY;
    return BSS_OK;
  }
  if (st != BSS_OK) return st;
  t.ms = ms / trials;
  t.drift = s.drift_rel_max;
  t.ok = std::isfinite(t.drift) && t.drift <= bound;
  return BSS_OK;
}

}  // namespace

extern "C" {

bss_status bss_autotune(const bss_instance *inst, const bss_options *base, double drift_bound, int32_t warmup_sweeps,
                        int32_t trial_sweeps, bss_tune_result *out) {
  if (!inst || !out || !(drift_bound > 0.0) || warmup_sweeps < 0 || trial_sweeps < 1) return BSS_E_INVALID_ARG;
  std::string why;
  if (!check_options(base, why)) return BSS_E_INVALID_ARG;
  bss_options opt;
  bss_options_default(&opt);
  if (base) opt = *base;
  opt.flags &= ~(BSS_FLAG_RECORD_TRACE | BSS_FLAG_REPLAY_TRACE | BSS_FLAG_PROFILE);
  opt.trace_sweeps = 0;
  opt.stream = nullptr;
  bss_status code;
  if (!valid_instance(*inst, why, code)) return code;
  const int N = inst->L * inst->L, Lam = (int)std::lround(inst->beta / inst->dtau);
  std::memset(out, 0, sizeof(*out));

  // equilibrated fields: FP64, short blocks
  std::vector<char> ck;
  {
    bss_options o0 = opt;
    o0.precision = BSS_PREC_FP64;
    o0.n_stab = std::min(4, Lam);
    o0.fp32_slices = 0;
    o0.workspace = nullptr;
    o0.workspace_bytes = 0;
    bss_ctx *c = nullptr;
    bss_instance in0 = *inst;
    in0.delay_k = in0.n_stab = 0;   // the options above decide
    bss_status st = create_impl(&in0, 1, &o0, &c);
    if (st != BSS_OK) return st;
    size_t n = 0;
    st = bss_sweep(c, warmup_sweeps, 0);
    if (st == BSS_OK) st = bss_save(c, nullptr, &n);
    if (st == BSS_OK) { ck.resize(n); st = bss_save(c, ck.data(), &n); }
    bss_destroy(c);
    if (st != BSS_OK) return st;
  }

  const int k_auto = auto_k(N);
  auto better = [](const Trial &a, const Trial &b) {   // a beats b
    if (a.ok != b.ok) return a.ok;
    if (!a.ok) return a.ns < b.ns;                     // nothing passes: the safest
    return a.ms < b.ms;
  };
  Trial best;
  bool have = false;
  int tried = 0;
  auto consider = [&](Trial t) -> bss_status {
    const bss_status st = run_trial(*inst, opt, ck, trial_sweeps, drift_bound, t);
    if (st != BSS_OK) return st;
    ++tried;
    if (!have || better(t, best)) { best = t; have = true; }
    return BSS_OK;
  };
  // 1. block length, FP64 slices only, up to a block condition estimate of
  // 1e12 (log cond of one slice: 2 lambda + 8 t dtau)
  const int ns_list[] = {2, 3, 4, 5, 6, 8, 10, 12, 16, 20};
  const double per = 2.0 * std::acosh(std::exp(0.5 * inst->dtau * inst->U)) + 8.0 * inst->t * inst->dtau;
  const double log_cap = std::log(1e12);
  std::vector<int> ns_try;
  for (int ns : ns_list)
    if (ns <= Lam && ns * per <= log_cap) ns_try.push_back(ns);
  if (ns_try.empty()) ns_try.push_back(std::max(1, std::min(Lam, (int)std::floor(log_cap / std::max(per, 1e-3)))));
  const int prec = opt.precision;
  opt.precision = BSS_PREC_FP64;   // phases 1 and 2 run every slice in FP64
  for (int ns : ns_try) {
    Trial t;
    t.k = k_auto; t.ns = ns; t.m32 = 0;
    const bss_status st = consider(t);
    if (st != BSS_OK) return st;
  }
  // 2. delay depth at that block length
  const int k_list_small[] = {1, 4, 8}, k_list_mid[] = {4, 8, 16}, k_list_big[] = {8, 16, 32};
  const int *kl = N <= 16 ? k_list_small : (N <= 64 ? k_list_mid : k_list_big);
  const int ns_best = best.ns;
  for (int q = 0; q < 3; ++q) {
    if (kl[q] == k_auto) continue;
    Trial t;
    t.k = kl[q]; t.ns = ns_best; t.m32 = 0;
    const bss_status st = consider(t);
    if (st != BSS_OK) return st;
  }
  // 3. FP32 slices at the end of each block
  opt.precision = prec;
  if (prec == BSS_PREC_MIXED && best.ok) {
    const int k_best = best.k;
    for (int m = 1; m <= ns_best; ++m) {
      Trial t;
      t.k = k_best; t.ns = ns_best; t.m32 = m;
      const bss_status st = run_trial(*inst, opt, ck, trial_sweeps, drift_bound, t);
      if (st != BSS_OK) return st;
      ++tried;
      if (!t.ok) break;
      if (better(t, best)) best = t;
    }
  }
  out->delay_k = best.k;
  out->n_stab = best.ns;
  out->fp32_slices = best.m32;
  out->precision = best.m32 > 0 ? BSS_PREC_MIXED : BSS_PREC_FP64;
  out->met_bound = best.ok ? 1 : 0;
  out->candidates = tried;
  out->ms_per_sweep = best.ms;
  out->drift_rel_max = best.drift;
  return BSS_OK;
}

void bss_destroy(bss_ctx *c) {
  if (!c) return;
  // everything finished first, then the graphs (and their events), then the
  // events and streams of direct launches, then the memory
  // (teardown: a failure here has nothing left to report to)
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &I : c->sh) {
    if (I.s) (void)hipStreamSynchronize(I.s);
    if (I.aux) (void)hipStreamSynchronize(I.aux);
  }
  destroy_graphs(c);
  for (auto &I : c->sh) {
    if (I.s) (void)hipStreamDestroy(I.s);
    if (I.aux) (void)hipStreamDestroy(I.aux);
    if (I.ev_main) (void)hipEventDestroy(I.ev_main);
    if (I.ev_left) (void)hipEventDestroy(I.ev_left);
  }
  for (auto &f : c->fam)
    for (auto &p : f.pending) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->own_mem && c->mem) (void)hipFree(c->mem);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *bss_status_string(bss_status s) {
  switch (s) {
    case BSS_OK: return "ok";
    case BSS_E_INVALID_ARG: return "invalid argument";
    case BSS_E_UNSUPPORTED: return "unsupported";
    case BSS_E_OUT_OF_MEMORY: return "out of memory";
    case BSS_E_DEVICE: return "device error";
    case BSS_E_NUMERICAL: return "numerical failure";
    case BSS_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char *bss_last_error(const bss_ctx *c) { return c ? c->last_error.c_str() : ""; }

}  // extern "C"
