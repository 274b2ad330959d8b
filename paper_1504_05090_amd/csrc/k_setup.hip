// Set-up and small elementwise kernels: kinetic exponentials, field
// initialisation, diagonal slice factors, identity stacks, counters.
#include "common.h"
#include "kernels.h"

namespace bss {

namespace {

// e^{-+dtau K} by plane waves: K is diagonalised by the lattice Fourier modes
// with eigenvalues eps_k = -2t(cos kx + cos ky), so
//   (e^{s K})_ij = (1/N) sum_k cos(k.(r_i - r_j)) e^{s eps_k}.
// Phases are reduced modulo L in integers before the cosine.
template <typename T>
__global__ void k_build_exp(int L, double t, double dtau, double *Em, double *Ep, T *Etm, T *Etp) {
  const int N = L * L;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const int dx = ((i % L) - (j % L) + L) % L, dy = ((i / L) - (j / L) + L) % L;
  double sm = 0.0, sp = 0.0;
  for (int my = 0; my < L; ++my)
    for (int mx = 0; mx < L; ++mx) {
      const double eps = -2.0 * t * (cospi(2.0 * mx / L) + cospi(2.0 * my / L));
      const double ph = cospi(2.0 * ((mx * dx + my * dy) % L) / L);
      sm += ph * exp(-dtau * eps);
      sp += ph * exp(dtau * eps);
    }
  sm /= N;
  sp /= N;
  Em[e] = sm;
  Ep[e] = sp;
  if (Etm) { Etm[e] = (T)sm; Etp[e] = (T)sp; }
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

hipError_t build_exp(int L, double t, double dtau, double *Em, double *Ep, void *Etm, void *Etp,
                     bool fp64, hipStream_t s) {
  const long n = (long)L * L * L * L;
  if (fp64 || !Etm)
    hipLaunchKernelGGL(k_build_exp<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, L, t, dtau, Em, Ep,
                       (double *)Etm, (double *)Etp);
  else
    hipLaunchKernelGGL(k_build_exp<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, L, t, dtau, Em, Ep,
                       (float *)Etm, (float *)Etp);
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
