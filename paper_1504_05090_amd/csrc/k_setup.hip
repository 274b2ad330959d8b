// Set-up and small elementwise kernels: kinetic exponentials, field
// initialisation, diagonal slice factors, identity stacks, counters.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {

// e^{-+dtau K} in closed form.  The hopping of eq. (1) on the periodic
// square lattice is K = -t (A_x + A_y) with commuting ring adjacencies, so
//   (e^{-s K})_ij = r(dx) r(dy),   r(d) = sum_w (sgn)^{n} I_n(2 s t),  n = |d + w L|,
// a sum over the periodic images of the one-dimensional free propagator
// (I_n: modified Bessel function of the first kind; sgn = +1 for e^{-dtau K},
// -1 for e^{+dtau K}).  Every term has the same sign for even L, so even the
// smallest entries (~1e-24 at 16 x 16) come out to full relative precision,
// which a plane-wave sum (absolute error ~1e-15) cannot give.
__device__ double bessel_i(int n, double x) {
  const double h = 0.5 * x;
  double term = 1.0;
  for (int j = 1; j <= n; ++j) term *= h / j;
  double sum = 0.0;
  for (int k = 0; k < 200 && term > 0.0; ++k) {
    sum += term;
    if (term < 1e-18 * sum) break;
    term *= h * h / ((double)(k + 1) * (double)(n + k + 1));
  }
  return sum;
}

__device__ double ring_propagator(int d, int L, double x, bool alternate) {
  double sum = 0.0;
  for (int w = 0; w <= 64; ++w) {
    double part = 0.0;
    const int np = d + w * L, nm = w > 0 ? (w * L - d) : -1;   // images +w and -w
    if (np <= 400) part += ((alternate && (np & 1)) ? -1.0 : 1.0) * bessel_i(np, x);
    if (nm >= 0 && nm <= 400) part += ((alternate && (nm & 1)) ? -1.0 : 1.0) * bessel_i(nm, x);
    sum += part;
    if (w > 0 && fabs(part) <= 1e-18 * fabs(sum)) break;
  }
  return sum;
}

__global__ void k_build_exp(int L, double t, double dtau, double *Em, double *Ep, float *Etm, float *Etp) {
  const int N = L * L;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const int dx = ((i % L) - (j % L) + L) % L, dy = ((i / L) - (j / L) + L) % L;
  const double x = 2.0 * dtau * t;
  const double sm = ring_propagator(dx, L, x, false) * ring_propagator(dy, L, x, false);
  const double sp = ring_propagator(dx, L, x, true) * ring_propagator(dy, L, x, true);
  Em[e] = sm;
  Ep[e] = sp;
  if (Etm) { Etm[e] = (float)sm; Etp[e] = (float)sp; }
}

__global__ void k_build_ring(int L, double t, double dtau, double *rm, double *rp, float *rtm, float *rtp) {
  const int d = threadIdx.x;
  if (d >= L) return;
  const double x = 2.0 * dtau * t;
  const double m = ring_propagator(d, L, x, false), p = ring_propagator(d, L, x, true);
  rm[d] = m;
  rp[d] = p;
  if (rtm) { rtm[d] = (float)m; rtp[d] = (float)p; }
}

// h[c][l][i] = +1 iff bit 63 of Philox word 0 at counter (0, l*N + i, 1, 0),
// key (seed + c, inst), is clear.
__global__ void k_init_field(int8_t *h, int chains, int Lam, int N, uint64_t seed, uint64_t inst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)Lam * N;
  if (e >= per * chains) return;
  const long c = e / per, pos = e % per;
  const uint64_t w = philox_word0(0, (uint64_t)pos, 1, 0, seed + (uint64_t)c, inst);
  h[e] = ((w >> 63) == 0) ? 1 : -1;
}

__global__ void k_slice_scales(const int8_t *h, int chains, int Lam, int N, int lo, int nq,
                               double elam, double emlam, double *out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)nq * N;
  if (e >= per * 2 * chains) return;
  const long mat = e / per, r = e % per;
  const int q = (int)(r / N), i = (int)(r % N);
  const int c = (int)(mat >> 1), spin = (int)(mat & 1);
  const int hv = h[((long)c * Lam + (lo - 1 + q)) * N + i];
  const bool up = (hv > 0) == (spin == 0);    // sigma * h > 0
  out[e] = up ? elam : emlam;
}

__global__ void k_scale_columns(const double *E, const double *d, long sd, double *P, int mats, int N) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)N * N;
  if (e >= nn * mats) return;
  const long m = e / nn, r = e % nn;
  P[e] = E[r] * d[m * sd + (r % N)];
}

__global__ void k_identity_udv(double *U, double *D, double *V, int mats, int N) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)N * N;
  if (e >= nn * mats) return;
  const long r = e % nn;
  const double v = ((r / N) == (r % N)) ? 1.0 : 0.0;
  U[e] = v;
  V[e] = v;
  if (r < N) D[(e / nn) * N + r] = 1.0;
}

template <typename T>
__global__ void k_copy_to_bulk(const double *src, T *dst, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (T)src[e];
}

__global__ void k_bump(int64_t *c) { c[0] += 1; }

__global__ void k_inv_big(const double *D, double *out, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = 1.0 / big_part(D[e]);
}

inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
}  // namespace

hipError_t build_exp(int L, double t, double dtau, double *Em, double *Ep, float *Etm, float *Etp, double *rm,
                     double *rp, float *rtm, float *rtp, hipStream_t s) {
  if (L < 1 || L > 1024) return hipErrorInvalidValue;
  const long n = (long)L * L * L * L;
  hipLaunchKernelGGL(k_build_exp, dim3(nblocks(n, 256)), dim3(256), 0, s, L, t, dtau, Em, Ep, Etm, Etp);
  hipLaunchKernelGGL(k_build_ring, dim3(1), dim3(1024), 0, s, L, t, dtau, rm, rp, rtm, rtp);
  return hipGetLastError();
}

hipError_t init_field(int8_t *h, int chains, int Lam, int N, uint64_t seed, uint64_t inst, hipStream_t s) {
  const long n = (long)chains * Lam * N;
  hipLaunchKernelGGL(k_init_field, dim3(nblocks(n, 256)), dim3(256), 0, s, h, chains, Lam, N, seed, inst);
  return hipGetLastError();
}

hipError_t slice_scales(const int8_t *h, int chains, int Lam, int N, int lo, int hi, double elam,
                        double emlam, double *out, hipStream_t s) {
  const int nq = hi - lo + 1;
  const long n = (long)2 * chains * nq * N;
  hipLaunchKernelGGL(k_slice_scales, dim3(nblocks(n, 256)), dim3(256), 0, s, h, chains, Lam, N, lo, nq,
                     elam, emlam, out);
  return hipGetLastError();
}

hipError_t scale_columns(const double *E, const double *d, long sd, double *P, int mats, int N, hipStream_t s) {
  const long n = (long)mats * N * N;
  hipLaunchKernelGGL(k_scale_columns, dim3(nblocks(n, 256)), dim3(256), 0, s, E, d, sd, P, mats, N);
  return hipGetLastError();
}

hipError_t set_identity_udv(double *U, double *D, double *V, int mats, int N, hipStream_t s) {
  const long n = (long)mats * N * N;
  hipLaunchKernelGGL(k_identity_udv, dim3(nblocks(n, 256)), dim3(256), 0, s, U, D, V, mats, N);
  return hipGetLastError();
}

hipError_t copy_to_bulk(const double *src, void *dst, long n, bool fp64, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_copy_to_bulk<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, src, (double *)dst, n);
  else
    hipLaunchKernelGGL(k_copy_to_bulk<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, src, (float *)dst, n);
  return hipGetLastError();
}

hipError_t bump_counter(int64_t *ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_bump, dim3(1), dim3(1), 0, s, ctr);
  return hipGetLastError();
}

hipError_t inv_big(const double *D, double *out, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_big, dim3(nblocks(n, 256)), dim3(256), 0, s, D, out, n);
  return hipGetLastError();
}

}  // namespace bss
