// Analysis of the sweep's output on the host (small data: a few hundred tau
// points per k): Trotter elimination (paper Sec. 3, "Trotter bias"), the
// Matsubara transform of eq. (5), the Dyson self-energy of eq. (6), the
// finite-size extrapolation in 1/L^2 (Sec. 3, last paragraph) and the
// correlation length of the spin correlation (Sec. 4).
//
// Readings where the paper is silent: cubic splines with not-a-knot ends
// through the slice grid tau_l = l dtau; the dtau -> 0 extrapolation is the
// constant term of a least-squares polynomial in dtau^2 of order
// min(2, grids - 1); eq. (5) is taken with e^{+i w_n tau}, the sign that agrees
// with eq. (6) under eq. (4)'s convention; the finite-size error bar is
// |linear - quadratic|; the correlation length comes from a least-squares fit
// of log|C| linear in the distance over 1 <= x <= L/2 along the axes.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "bssqmc.h"

namespace {

typedef std::complex<double> cplx;

// Cubic spline with not-a-knot ends through (x_i, y_i), i = 0..n: the slopes
// s_i solve the tridiagonal system of C2 continuity (rows 1..n-1) and of a
// continuous third derivative at x_1 and x_{n-1} (rows 0 and n), by Gaussian
// elimination with partial pivoting (one extra superdiagonal of fill).
struct Spline {
  std::vector<double> x, y, s;
  bool init(const double *xs, const double *ys, int npts) {
    const int n = npts - 1;
    if (n < 1) return false;
    x.assign(xs, xs + npts);
    y.assign(ys, ys + npts);
    s.assign(npts, 0.0);
    std::vector<double> h(n), d(n);
    for (int i = 0; i < n; ++i) {
      h[i] = x[i + 1] - x[i];
      if (!(h[i] > 0.0)) return false;
      d[i] = (y[i + 1] - y[i]) / h[i];
    }
    if (n == 1) { s[0] = s[1] = d[0]; return true; }
    if (n == 2) {   // one parabola through the three points
      const double c = (d[1] - d[0]) / (x[2] - x[0]);
      s[0] = d[0] - c * h[0];
      s[1] = d[0] + c * h[0];
      s[2] = d[1] + c * h[1];
      return true;
    }
    // rows: sub[i] s_{i-1} + dia[i] s_i + sup[i] s_{i+1} = b[i]
    std::vector<double> sub(npts, 0.0), dia(npts, 0.0), sup(npts, 0.0), b(npts, 0.0), sup2(npts, 0.0);
    {
      const double w = h[0] + h[1];
      dia[0] = h[1];
      sup[0] = w;
      b[0] = ((h[0] + 2.0 * w) * h[1] * d[0] + h[0] * h[0] * d[1]) / w;
    }
    for (int i = 1; i < n; ++i) {
      sub[i] = h[i];
      dia[i] = 2.0 * (h[i - 1] + h[i]);
      sup[i] = h[i - 1];
      b[i] = 3.0 * (h[i] * d[i - 1] + h[i - 1] * d[i]);
    }
    {
      const double w = h[n - 2] + h[n - 1];
      sub[n] = w;
      dia[n] = h[n - 2];
      b[n] = (h[n - 1] * h[n - 1] * d[n - 2] + (2.0 * w + h[n - 1]) * h[n - 2] * d[n - 1]) / w;
    }
    // forward elimination with row swaps between i and i + 1
    for (int i = 0; i < n; ++i) {
      if (std::fabs(sub[i + 1]) > std::fabs(dia[i])) {
        std::swap(dia[i], sub[i + 1]);
        std::swap(sup[i], dia[i + 1]);
        std::swap(sup2[i], sup[i + 1]);
        std::swap(b[i], b[i + 1]);
      }
      const double f = sub[i + 1] / dia[i];
      dia[i + 1] -= f * sup[i];
      sup[i + 1] -= f * sup2[i];
      b[i + 1] -= f * b[i];
      sub[i + 1] = 0.0;
    }
    for (int i = n; i >= 0; --i) {
      double v = b[i];
      if (i + 1 <= n) v -= sup[i] * s[i + 1];
      if (i + 2 <= n) v -= sup2[i] * s[i + 2];
      s[i] = v / dia[i];
    }
    return true;
  }
  // p(t) = y_i + s_i u + c2 u^2 + c3 u^3 on [x_i, x_{i+1}], u = t - x_i
  void coef(int i, double &a, double &b, double &c2, double &c3) const {
    const double h = x[i + 1] - x[i], d = (y[i + 1] - y[i]) / h;
    a = y[i];
    b = s[i];
    c2 = (3.0 * d - 2.0 * s[i] - s[i + 1]) / h;
    c3 = (s[i] + s[i + 1] - 2.0 * d) / (h * h);
  }
  int interval(double t) const {
    int lo = 0, hi = (int)x.size() - 2;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (x[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  double operator()(double t) const {
    const int i = interval(t);
    double a, b, c2, c3;
    coef(i, a, b, c2, c3);
    const double u = t - x[i];
    return a + u * (b + u * (c2 + u * c3));
  }
};

// least squares V c = y (A x P, A >= P, small) by Householder QR; returns c
bool lstsq(std::vector<double> V, int A, int P, std::vector<double> y, std::vector<double> &c) {
  for (int j = 0; j < P; ++j) {
    double nrm = 0.0;
    for (int i = j; i < A; ++i) nrm += V[i * P + j] * V[i * P + j];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = V[j * P + j] > 0 ? -nrm : nrm;
    std::vector<double> v(A, 0.0);
    for (int i = j; i < A; ++i) v[i] = V[i * P + j];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < A; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int q = j; q < P; ++q) {
      double w = 0.0;
      for (int i = j; i < A; ++i) w += v[i] * V[i * P + q];
      w = 2.0 * w / vv;
      for (int i = j; i < A; ++i) V[i * P + q] -= w * v[i];
    }
    double w = 0.0;
    for (int i = j; i < A; ++i) w += v[i] * y[i];
    w = 2.0 * w / vv;
    for (int i = j; i < A; ++i) y[i] -= w * v[i];
  }
  c.assign(P, 0.0);
  for (int j = P - 1; j >= 0; --j) {
    double v = y[j];
    for (int q = j + 1; q < P; ++q) v -= V[j * P + q] * c[q];
    if (V[j * P + j] == 0.0) return false;
    c[j] = v / V[j * P + j];
  }
  return true;
}

// I_k = int_0^h u^k e^{z u} du, k = 0..3: power series for |z h| <= 1/2,
// else the upward recursion I_k = (h^k e^{z h} - k I_{k-1}) / z
void moments(cplx z, double h, cplx I[4]) {
  if (std::abs(z) * h <= 0.5) {
    cplx zm(1.0, 0.0);
    double fact = 1.0;
    for (int k = 0; k < 4; ++k) I[k] = 0.0;
    for (int m = 0; m < 40; ++m) {
      for (int k = 0; k < 4; ++k) I[k] += zm * std::pow(h, m + k + 1) / (fact * (m + k + 1));
      zm *= z;
      fact *= (m + 1);
      if (std::abs(zm) * std::pow(h, m + 1) / fact < 1e-18 * h) break;
    }
    return;
  }
  const cplx e = std::exp(z * h);
  I[0] = (e - 1.0) / z;
  double hk = 1.0;
  for (int k = 1; k < 4; ++k) {
    hk *= h;
    I[k] = (hk * e - (double)k * I[k - 1]) / z;
  }
}

bool finite_all(const double *v, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

extern "C" {

bss_status bss_trotter_extrapolate(int32_t n_grids, const double *dtau, double beta, const double *const *G,
                                   int32_t n_cols, int32_t n_out, const double *tau_out, double *out) {
  if (n_grids < 2 || !dtau || !G || n_cols < 1 || n_out < 1 || !tau_out || !out || !(beta > 0.0))
    return BSS_E_INVALID_ARG;
  std::vector<int> lam(n_grids);
  for (int a = 0; a < n_grids; ++a) {
    if (!(dtau[a] > 0.0) || !G[a]) return BSS_E_INVALID_ARG;
    const double r = beta / dtau[a];
    lam[a] = (int)std::lround(r);
    if (lam[a] < 1 || std::fabs(r - lam[a]) > 1e-9 * r) return BSS_E_INVALID_ARG;
    if (!finite_all(G[a], (long)(lam[a] + 1) * n_cols)) return BSS_E_INVALID_ARG;
  }
  for (int m = 0; m < n_out; ++m)
    if (!(tau_out[m] >= 0.0 && tau_out[m] <= beta)) return BSS_E_INVALID_ARG;
  const int P = std::min(2, n_grids - 1) + 1;
  std::vector<double> V((size_t)n_grids * P);
  for (int a = 0; a < n_grids; ++a) {
    const double x = dtau[a] * dtau[a];
    double p = 1.0;
    for (int j = 0; j < P; ++j) { V[a * P + j] = p; p *= x; }
  }
  // aligned[a][m][col]
  std::vector<double> aligned((size_t)n_grids * n_out * n_cols);
  for (int a = 0; a < n_grids; ++a) {
    std::vector<double> tau(lam[a] + 1), col(lam[a] + 1);
    for (int l = 0; l <= lam[a]; ++l) tau[l] = l * dtau[a];
    for (int k = 0; k < n_cols; ++k) {
      for (int l = 0; l <= lam[a]; ++l) col[l] = G[a][(size_t)l * n_cols + k];
      Spline sp;
      if (!sp.init(tau.data(), col.data(), lam[a] + 1)) return BSS_E_INVALID_ARG;
      for (int m = 0; m < n_out; ++m) aligned[((size_t)a * n_out + m) * n_cols + k] = sp(tau_out[m]);
    }
  }
  std::vector<double> y(n_grids), c;
  for (int m = 0; m < n_out; ++m)
    for (int k = 0; k < n_cols; ++k) {
      for (int a = 0; a < n_grids; ++a) y[a] = aligned[((size_t)a * n_out + m) * n_cols + k];
      if (!lstsq(V, n_grids, P, y, c)) return BSS_E_NUMERICAL;
      out[(size_t)m * n_cols + k] = c[0];
    }
  return BSS_OK;
}

bss_status bss_matsubara(int32_t n_tau, const double *tau, const double *G, double beta, int32_t n_freq,
                         double *out_re_im) {
  if (n_tau < 2 || !tau || !G || n_freq < 1 || !out_re_im || !(beta > 0.0)) return BSS_E_INVALID_ARG;
  if (std::fabs(tau[0]) > 1e-12 * beta || std::fabs(tau[n_tau - 1] - beta) > 1e-12 * beta) return BSS_E_INVALID_ARG;
  if (!finite_all(G, n_tau) || !finite_all(tau, n_tau)) return BSS_E_INVALID_ARG;
  Spline sp;
  if (!sp.init(tau, G, n_tau)) return BSS_E_INVALID_ARG;
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < n_freq; ++n) {
    const cplx z(0.0, (2.0 * n + 1.0) * pi / beta);
    cplx acc = 0.0;
    for (int i = 0; i + 1 < n_tau; ++i) {
      double a, b, c2, c3;
      sp.coef(i, a, b, c2, c3);
      cplx I[4];
      moments(z, tau[i + 1] - tau[i], I);
      acc += std::exp(z * tau[i]) * (a * I[0] + b * I[1] + c2 * I[2] + c3 * I[3]);
    }
    out_re_im[2 * n] = acc.real();
    out_re_im[2 * n + 1] = acc.imag();
  }
  return BSS_OK;
}

bss_status bss_dyson(int32_t n_freq, double beta, double eps_k, double mu, const double *G_re_im,
                     double *sigma_re_im) {
  if (n_freq < 1 || !G_re_im || !sigma_re_im || !(beta > 0.0)) return BSS_E_INVALID_ARG;
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < n_freq; ++n) {
    const cplx g(G_re_im[2 * n], G_re_im[2 * n + 1]);
    if (g == 0.0 || !std::isfinite(g.real()) || !std::isfinite(g.imag())) return BSS_E_NUMERICAL;
    const cplx sig = cplx(mu - eps_k, (2.0 * n + 1.0) * pi / beta) - 1.0 / g;
    sigma_re_im[2 * n] = sig.real();
    sigma_re_im[2 * n + 1] = sig.imag();
  }
  return BSS_OK;
}

bss_status bss_finite_size_extrapolate(int32_t n_L, const int32_t *L, int32_t n_vals, const double *values,
                                       double *value, double *err, double *lin, double *quad) {
  if (n_L < 3 || !L || n_vals < 1 || !values || !value || !err) return BSS_E_INVALID_ARG;
  for (int a = 0; a < n_L; ++a)
    if (L[a] < 1) return BSS_E_INVALID_ARG;
  if (!finite_all(values, (long)n_L * n_vals)) return BSS_E_INVALID_ARG;
  std::vector<double> V1((size_t)n_L * 2), V2((size_t)n_L * 3);
  for (int a = 0; a < n_L; ++a) {
    const double x = 1.0 / ((double)L[a] * L[a]);
    V1[a * 2] = 1.0; V1[a * 2 + 1] = x;
    V2[a * 3] = 1.0; V2[a * 3 + 1] = x; V2[a * 3 + 2] = x * x;
  }
  std::vector<double> y(n_L), c1, c2;
  for (int v = 0; v < n_vals; ++v) {
    for (int a = 0; a < n_L; ++a) y[a] = values[(size_t)a * n_vals + v];
    if (!lstsq(V1, n_L, 2, y, c1) || !lstsq(V2, n_L, 3, y, c2)) return BSS_E_NUMERICAL;
    value[v] = 0.5 * (c1[0] + c2[0]);
    err[v] = std::fabs(c1[0] - c2[0]);
    if (lin) lin[v] = c1[0];
    if (quad) quad[v] = c2[0];
  }
  return BSS_OK;
}

bss_status bss_correlation_length(int32_t L, const double *C, double *xi, double *amplitude) {
  if (L < 4 || !C || !xi) return BSS_E_INVALID_ARG;
  const int n = L / 2;
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (int x = 1; x <= n; ++x) {
    const double c = 0.5 * (std::fabs(C[x]) + std::fabs(C[(size_t)x * L]));
    if (!(c > 0.0) || !std::isfinite(c)) return BSS_E_NUMERICAL;
    const double ly = std::log(c);
    sx += x; sy += ly; sxx += (double)x * x; sxy += x * ly;
  }
  const double den = n * sxx - sx * sx;
  const double slope = (n * sxy - sx * sy) / den, icpt = (sy - slope * sx) / n;
  if (!(slope < 0.0)) return BSS_E_NUMERICAL;
  *xi = -1.0 / slope;
  if (amplitude) *amplitude = std::exp(icpt);
  return BSS_OK;
}

}  // extern "C"
