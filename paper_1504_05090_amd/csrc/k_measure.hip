// Measurement kernels (FP64): double occupancy, the momentum-resolved
// time-displaced Green function and the real-space spin correlation,
// accumulated per chain in blocked bins.
//
//   D = (1/N) sum_i (1 - G_up,ii)(1 - G_dn,ii)        (Wick, spins decouple per field)
//   C(r) = (1/N) sum_i <S^z_i S^z_{i+r}>,  S^z = (n_up - n_dn)/2  (paper Sec. 4, Fig. 5):
//     per field <S^z_i S^z_j> = [m_i m_j + sum_s (delta_ij G_s,ii - G_s,ji G_s,ij)] / 4,
//     m_i = <n_i,up> - <n_i,dn> = G_dn,ii - G_up,ii
//   G(tau_l, k) = -1/2 sum_sigma (1/N) sum_ij cos(k.(r_i - r_j)) G_sigma,ij(tau_l, 0)
// The second is evaluated through the lattice-averaged g(delta) =
// (1/N) sum_i G_{i+delta, i}, then G(tau_l, k) = -1/2 sum_delta cos(k.delta) g(delta)
// with g summed over both spins.
#include "common.h"
#include "kernels.h"
#include "measure.h"

namespace bss {

namespace {

// Start a measurement: pick the bin of measurement n = count[c]; when all
// nbins bins are full, merge neighbours pairwise and double the bin size.
__global__ void k_meas_begin(MeasState ms, int chains) {
  const int c = blockIdx.x;
  if (c >= chains) return;
  int64_t n = ms.count[c];
  int64_t bs = ms.binsize[c];
  __shared__ int merge;
  if (threadIdx.x == 0) merge = (n / bs) >= ms.nbins;
  __syncthreads();
  if (merge) {
    const long per_g = ms.glen;
    double *gb = ms.gk + (long)c * ms.nbins_g * per_g;
    double *db = ms.docc + (long)c * ms.nbins;
    if (ms.nbins_g == ms.nbins) {
      // per offset, sequentially in the bin index: bin b is read (as 2b' or
      // 2b'+1 for b' = b/2 < b) before it is overwritten
      for (long off = threadIdx.x; off < per_g; off += blockDim.x) {
        for (int bin = 0; bin < ms.nbins / 2; ++bin)
          gb[bin * per_g + off] = gb[(2 * bin) * per_g + off] + gb[(2 * bin + 1) * per_g + off];
        for (int bin = ms.nbins / 2; bin < ms.nbins; ++bin) gb[bin * per_g + off] = 0.0;
      }
      double *sb = ms.sc + (long)c * ms.nbins_g * ms.sclen;
      for (long off = threadIdx.x; off < ms.sclen; off += blockDim.x) {
        for (int bin = 0; bin < ms.nbins / 2; ++bin)
          sb[bin * ms.sclen + off] = sb[(2 * bin) * ms.sclen + off] + sb[(2 * bin + 1) * ms.sclen + off];
        for (int bin = ms.nbins / 2; bin < ms.nbins; ++bin) sb[bin * ms.sclen + off] = 0.0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int b = 0; b < ms.nbins / 2; ++b) db[b] = db[2 * b] + db[2 * b + 1];
      for (int b = ms.nbins / 2; b < ms.nbins; ++b) db[b] = 0.0;
      ms.binsize[c] = bs * 2;
    }
    bs *= 2;
  }
  if (threadIdx.x == 0) ms.cur[c] = (int)(n / bs);
}

__global__ void k_meas_end(MeasState ms, int chains) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < chains) ms.count[c] += 1;
}

__global__ __launch_bounds__(256) void k_meas_docc(MeasState ms, const double *Gf, int N) {
  __shared__ double red[16];
  const int c = blockIdx.x;
  const double *gu = Gf + (2L * c) * N * N, *gd = gu + (long)N * N;
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    s += (1.0 - gu[(long)i * N + i]) * (1.0 - gd[(long)i * N + i]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) ms.docc[(long)c * ms.nbins + ms.cur[c]] += s / N;
}

// One chain per block: g(delta) summed over spins, then its cosine transform,
// added to the slice-l row of the chain's current bin.
//  - g(delta) = (1/N) sum_r G_{r, r - delta}: each thread owns displacements
//    delta and walks the rows r, so at each step the lanes of a wavefront
//    read within one row of G (the lattice difference r - delta permutes the
//    columns);
//  - the transform is separable, sum_delta cos(k.delta) g(delta) =
//    Re sum_dy e^{i ky dy} sum_dx e^{i kx dx} g(dx, dy), taken as two passes of
//    L terms with cos and sin of 2 pi m / L from a table.
__global__ __launch_bounds__(256) void k_meas_gk(MeasState ms, const double *Gt, int L, int l) {
  extern __shared__ double sh[];
  const int N = L * L, c = blockIdx.x;
  double *gd = sh, *hre = sh + N, *him = sh + 2 * N, *cs = sh + 3 * N, *sn = cs + L;
  const double *g0 = Gt + (2L * c) * N * N, *g1 = g0 + (long)N * N;
  for (int m = threadIdx.x; m < L; m += blockDim.x) {
    cs[m] = cospi(2.0 * m / L);
    sn[m] = sinpi(2.0 * m / L);
  }
  for (int dlt = threadIdx.x; dlt < N; dlt += blockDim.x) {
    const int dx = dlt % L, dy = dlt / L;
    double s = 0.0;
    for (int r = 0; r < N; ++r) {
      const int col = ((r % L) - dx + L) % L + L * (((r / L) - dy + L) % L);
      s += g0[(long)r * N + col] + g1[(long)r * N + col];
    }
    gd[dlt] = s / N;
  }
  __syncthreads();
  // h(mx, dy) = sum_dx e^{2 pi i mx dx / L} g(dx, dy)
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    const int mx = e % L, dy = e / L;
    double re = 0.0, im = 0.0;
    for (int dx = 0; dx < L; ++dx) {
      const int ph = (mx * dx) % L;
      re += cs[ph] * gd[dx + L * dy];
      im += sn[ph] * gd[dx + L * dy];
    }
    hre[e] = re;
    him[e] = im;
  }
  __syncthreads();
  double *out = ms.gk + ((long)c * ms.nbins_g + (ms.nbins_g == 1 ? 0 : ms.cur[c])) * ms.glen + (long)l * N;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const int mx = k % L, my = k / L;
    double s = 0.0;
    for (int dy = 0; dy < L; ++dy) {
      const int ph = (my * dy) % L;
      s += cs[ph] * hre[mx + L * dy] - sn[ph] * him[mx + L * dy];
    }
    out[k] += -0.5 * s;
  }
}

// One chain per block: the local moments in LDS, then one displacement r
// per thread summed over the sites i (j = i + r with periodic wrap).
__global__ __launch_bounds__(256) void k_meas_sc(MeasState ms, const double *Gf, int L) {
  extern __shared__ double mom[];   // [N] m_i = G_dn,ii - G_up,ii
  const int N = L * L, c = blockIdx.x;
  const double *gu = Gf + (2L * c) * N * N, *gd = gu + (long)N * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) mom[i] = gd[(long)i * N + i] - gu[(long)i * N + i];
  __syncthreads();
  double *out = ms.sc + ((long)c * ms.nbins_g + (ms.nbins_g == 1 ? 0 : ms.cur[c])) * ms.sclen;
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const int dx = r % L, dy = r / L;
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
      const int j = ((i % L) + dx) % L + L * (((i / L) + dy) % L);
      s += mom[i] * mom[j] - gu[(long)j * N + i] * gu[(long)i * N + j] - gd[(long)j * N + i] * gd[(long)i * N + j];
      if (j == i) s += gu[(long)i * N + i] + gd[(long)i * N + i];
    }
    out[r] += 0.25 * s / N;
  }
}
}  // namespace

hipError_t meas_begin(const MeasState &ms, int chains, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_begin, dim3(chains), dim3(256), 0, s, ms, chains);
  return hipGetLastError();
}
hipError_t meas_end(const MeasState &ms, int chains, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_end, dim3((chains + 255) / 256), dim3(256), 0, s, ms, chains);
  return hipGetLastError();
}
hipError_t meas_docc(const MeasState &ms, const double *Gf, int chains, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_docc, dim3(chains), dim3(256), 0, s, ms, Gf, N);
  return hipGetLastError();
}
hipError_t meas_sc(const MeasState &ms, const double *Gf, int chains, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_sc, dim3(chains), dim3(256), sizeof(double) * L * L, s, ms, Gf, L);
  return hipGetLastError();
}
hipError_t meas_gk(const MeasState &ms, const double *Gt, int chains, int L, int l, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_gk, dim3(chains), dim3(256), sizeof(double) * (3 * L * L + 2 * L), s, ms, Gt, L, l);
  return hipGetLastError();
}

}  // namespace bss
