// Maximum-entropy regularisation of G(tau) on the host (Sec. 3, Trotter-bias
// paragraph, with eq. (4)): a spectral function A(w) >= 0 is fitted to
// G(tau) through eq. (4), and only the G(tau) it gives back is used further.
//
// Readings where the paper is silent (the entry points' documentation
// repeats them): trapezoid weights q_j on a caller-given increasing w grid,
// so eq. (4) reads G_i = -sum_j q_j K(tau_i, w_j) A_j with K = e^{-w tau} /
// (1 + e^{-w beta}); chi^2 with one standard error per tau point; the
// Shannon-Jaynes entropy S = sum_j q_j (A_j - m_j - A_j ln(A_j/m_j)) relative
// to a caller-given default model m > 0; A minimises Q = chi^2/2 - alpha S at
// a fixed alpha, or at the historic alpha where chi^2 = number of tau points.
//
// Algorithm (Bryan's singular-space method): in the masses a_j = q_j A_j the
// stationarity condition of Q reads alpha ln(a/mu) = -C^T (C a - d), with
// C_ij = -K_ij / sigma_i, d_i = G_i / sigma_i and mu_j = q_j m_j, so ln(a/mu)
// lies in the row space of C.  With the thin SVD C^T = U Sigma V^T (one-sided
// Jacobi, singular values below max(n, M) eps sigma_max dropped) the unknown is
// u in a = mu exp(U u), s = rank(C) numbers instead of M.  The stationarity
// condition alpha u + Sigma V^T (C a - d) = 0 is solved by Newton's method
// (its Jacobian has eigenvalues >= alpha), with backtracking on Q itself
// (the Newton step descends on it); once the Newton step is at most 1e-8 the full step is taken and
// the iteration ends (the quadratic phase leaves an error of order 1e-16).
// The historic alpha is the root of chi^2(alpha) - n in ln alpha (chi^2
// grows with alpha), bracketed by decades downwards from alpha = 1e12 to at
// most 1e-8 and found by regula falsi with the Illinois modification, each
// solve starting from the nearest solution already found.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bssqmc.h"

namespace {

double kern(double tau, double w, double beta) {
  return w >= 0.0 ? std::exp(-w * tau) / (1.0 + std::exp(-w * beta))
                  : std::exp(w * (beta - tau)) / (std::exp(w * beta) + 1.0);
}

void trapezoid(const double *w, int M, std::vector<double> &q) {
  q.assign(M, 0.0);
  for (int j = 0; j + 1 < M; ++j) {
    const double h = 0.5 * (w[j + 1] - w[j]);
    q[j] += h;
    q[j + 1] += h;
  }
}

// Solve J x = b (J s x s, row-major, overwritten; b in x) by Gaussian
// elimination with partial pivoting; false if J is singular to working
// precision.
bool lu_solve(std::vector<double> &J, int s, std::vector<double> &x) {
  for (int c = 0; c < s; ++c) {
    int p = c;
    for (int i = c + 1; i < s; ++i)
      if (std::fabs(J[(size_t)i * s + c]) > std::fabs(J[(size_t)p * s + c])) p = i;
    if (!(std::fabs(J[(size_t)p * s + c]) > 0.0) || !std::isfinite(J[(size_t)p * s + c])) return false;
    if (p != c) {
      for (int k = 0; k < s; ++k) std::swap(J[(size_t)p * s + k], J[(size_t)c * s + k]);
      std::swap(x[p], x[c]);
    }
    for (int i = c + 1; i < s; ++i) {
      const double f = J[(size_t)i * s + c] / J[(size_t)c * s + c];
      if (f == 0.0) continue;
      for (int k = c; k < s; ++k) J[(size_t)i * s + k] -= f * J[(size_t)c * s + k];
      x[i] -= f * x[c];
    }
  }
  for (int i = s - 1; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < s; ++k) v -= J[(size_t)i * s + k] * x[k];
    x[i] = v / J[(size_t)i * s + i];
  }
  return true;
}

struct Mem {
  int n, M, s;
  std::vector<double> C;    // [n][M]  -K_ij / sigma_i
  std::vector<double> d;    // [n]     G_i / sigma_i
  std::vector<double> mu;   // [M]     q_j m_j
  std::vector<double> U;    // [M][s]  left singular vectors of C^T (columns)
  // per-iterate work
  std::vector<double> z, a, r, h;
  double Qscale = 0;   // sum of the magnitudes of Q's terms (its rounding is ~eps Qscale)

  // Thin SVD of C^T (M x n) by one-sided Jacobi on its n columns: rotate
  // pairs of columns until all are orthogonal to working precision; the
  // column norms are the singular values and the normalised columns U.
  void svd() {
    std::vector<double> X((size_t)n * M);   // column k of C^T is row k of C
    std::memcpy(X.data(), C.data(), sizeof(double) * X.size());
    const double eps = 2.220446049250313e-16;
    for (int sweep = 0; sweep < 60; ++sweep) {
      bool rotated = false;
      for (int p = 0; p < n; ++p)
        for (int qc = p + 1; qc < n; ++qc) {
          double *xp = &X[(size_t)p * M], *xq = &X[(size_t)qc * M];
          double app = 0, aqq = 0, apq = 0;
          for (int j = 0; j < M; ++j) { app += xp[j] * xp[j]; aqq += xq[j] * xq[j]; apq += xp[j] * xq[j]; }
          if (std::fabs(apq) <= eps * std::sqrt(app * aqq) || apq == 0.0) continue;
          rotated = true;
          const double zeta = (aqq - app) / (2.0 * apq);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
          for (int j = 0; j < M; ++j) {
            const double u = xp[j], v = xq[j];
            xp[j] = c * u - sn * v;
            xq[j] = sn * u + c * v;
          }
        }
      if (!rotated) break;
    }
    std::vector<std::pair<double, int>> sv(n);
    for (int k = 0; k < n; ++k) {
      double nrm = 0;
      for (int j = 0; j < M; ++j) nrm += X[(size_t)k * M + j] * X[(size_t)k * M + j];
      sv[k] = {std::sqrt(nrm), k};
    }
    std::sort(sv.begin(), sv.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
      return x.first > y.first;
    });
    const double cut = sv[0].first * std::max(n, M) * eps;
    s = 0;
    while (s < n && sv[s].first > cut) ++s;
    U.assign((size_t)M * s, 0.0);
    for (int k = 0; k < s; ++k)
      for (int j = 0; j < M; ++j) U[(size_t)j * s + k] = X[(size_t)sv[k].second * M + j] / sv[k].first;
  }

  // a = mu exp(U u), r = C a - d, Q; false if a leaves the representable
  // positive range or Q is not finite.
  bool eval(const std::vector<double> &u, double alpha, double &Q) {
    z.assign(M, 0.0);
    a.resize(M);
    double ent = 0.0, ent_mag = 0.0;
    for (int j = 0; j < M; ++j) {
      double v = 0;
      for (int k = 0; k < s; ++k) v += U[(size_t)j * s + k] * u[k];
      z[j] = v;
      a[j] = mu[j] * std::exp(v);
      if (!(a[j] > 1e-290) || !std::isfinite(a[j])) return false;
      ent += a[j] - mu[j] - a[j] * v;
      ent_mag += a[j] + mu[j] + std::fabs(a[j] * v);
    }
    r.resize(n);
    double chi2 = 0.0;
    for (int i = 0; i < n; ++i) {
      double v = -d[i];
      for (int j = 0; j < M; ++j) v += C[(size_t)i * M + j] * a[j];
      r[i] = v;
      chi2 += v * v;
    }
    Q = 0.5 * chi2 - alpha * ent;
    Qscale = 0.5 * chi2 + alpha * ent_mag;
    return std::isfinite(Q);
  }

  double chi2() const {
    double c = 0;
    for (int i = 0; i < n; ++i) c += r[i] * r[i];
    return c;
  }

  // Stationary point of Q at alpha from u (in place): the root of
  // F(u) = U^T (C^T r + alpha U u) = alpha u + Sigma V^T r (U^T C^T = Sigma V^T
  // holds also for the truncated SVD), whose Jacobian
  // J = alpha I + (C U)^T C diag(a) U = alpha I + Sigma^2 U^T diag(a) U has
  // eigenvalues >= alpha, so the Newton step du = -J^-1 F is defined for
  // every a > 0.  It descends on Q itself: with T = U^T diag(a) U (SPD) the
  // gradient of Q in u is T F and J = alpha I + Sigma^2 T, so
  // grad Q . du = -F^T (alpha T^-1 + Sigma^2)^-1 F < 0; and the only
  // stationary point of Q in u is the minimiser.  The step is therefore
  // backtracked on Q (Armijo, within Q's rounding), which unlike |F|^2 does
  // not stall where the exponential makes F far from linear.  false: no
  // convergence.
  bool solve(double alpha, std::vector<double> &u) {
    double Q;
    if (!eval(u, alpha, Q)) return false;
    if (R.empty()) {   // C U, fixed for the problem
      R.assign((size_t)n * s, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < M; ++j) {
          const double c = C[(size_t)i * M + j];
          for (int k = 0; k < s; ++k) R[(size_t)i * s + k] += c * U[(size_t)j * s + k];
        }
    }
    std::vector<double> F(s), Fn(s), J((size_t)s * s), P((size_t)n * s), du(s), un(s);
    residual_F(alpha, F);
    double phi = 0.5 * dot(F, F), Qc = Q, Qsc = Qscale;
    for (int it = 0; it < 500; ++it) {
      // J = alpha I + R^T P, P = C diag(a) U
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < s; ++k) {
          double v = 0;
          for (int j = 0; j < M; ++j) v += C[(size_t)i * M + j] * a[j] * U[(size_t)j * s + k];
          P[(size_t)i * s + k] = v;
        }
      for (int k = 0; k < s; ++k)
        for (int l = 0; l < s; ++l) {
          double v = k == l ? alpha : 0.0;
          for (int i = 0; i < n; ++i) v += R[(size_t)i * s + k] * P[(size_t)i * s + l];
          J[(size_t)k * s + l] = v;
        }
      for (int k = 0; k < s; ++k) du[k] = -F[k];
      if (!lu_solve(J, s, du)) return false;
      double step = 0;
      for (int k = 0; k < s; ++k) step = std::max(step, std::fabs(du[k]));
      if (step <= 1e-8) {
        // quadratic phase: the full step leaves an error of O(step^2); it is
        // kept unless it makes the residual worse (rounding level)
        for (int k = 0; k < s; ++k) un[k] = u[k] + du[k];
        bool keep = eval(un, alpha, Q);
        if (keep) {
          residual_F(alpha, Fn);
          keep = 0.5 * dot(Fn, Fn) <= phi;
        }
        if (keep) u = un;
        else if (!eval(u, alpha, Q)) return false;
        return true;
      }
      // slope of Q along du: (U F)^T diag(a) (U du), a at the current u
      double slope = 0.0;
      for (int j = 0; j < M; ++j) {
        double uf = 0.0, ud = 0.0;
        for (int k = 0; k < s; ++k) {
          uf += U[(size_t)j * s + k] * F[k];
          ud += U[(size_t)j * s + k] * du[k];
        }
        slope += a[j] * uf * ud;
      }
      slope = std::min(slope, 0.0);
      double t = 1.0;
      bool accepted = false;
      for (; t >= 1e-30; t *= 0.5) {
        for (int k = 0; k < s; ++k) un[k] = u[k] + t * du[k];
        if (!eval(un, alpha, Q)) continue;
        const double tol = 1e-13 * std::max(Qsc, Qscale);
        if (Q <= Qc + 1e-4 * t * slope + tol) { accepted = true; break; }
      }
      if (!accepted) return false;
      u = un;
      Qc = Q;
      Qsc = Qscale;
      residual_F(alpha, F);
      phi = 0.5 * dot(F, F);
    }
    return false;
  }

  std::vector<double> R;    // [n][s] C U

  // F = U^T (C^T r + alpha z) from the current iterate
  void residual_F(double alpha, std::vector<double> &F) {
    h.assign(M, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < M; ++j) h[j] += C[(size_t)i * M + j] * r[i];
    for (int j = 0; j < M; ++j) h[j] += alpha * z[j];
    for (int k = 0; k < s; ++k) {
      double v = 0;
      for (int j = 0; j < M; ++j) v += U[(size_t)j * s + k] * h[j];
      F[k] = v;
    }
  }

  static double dot(const std::vector<double> &x, const std::vector<double> &y) {
    double v = 0;
    for (size_t i = 0; i < x.size(); ++i) v += x[i] * y[i];
    return v;
  }
};

bool finite_all(const double *x, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

extern "C" {

bss_status bss_mem_spectrum(int32_t n_tau, const double *tau, const double *G, const double *sigma, double beta,
                            int32_t n_omega, const double *omega, const double *model, double alpha, double *A,
                            double *alpha_out, double *chi2_out) {
  if (n_tau < 2 || n_omega < 2 || !tau || !G || !sigma || !omega || !model || !A || !(beta > 0.0) ||
      !std::isfinite(beta) || std::isnan(alpha) || std::isinf(alpha))
    return BSS_E_INVALID_ARG;
  if (!finite_all(tau, n_tau) || !finite_all(G, n_tau) || !finite_all(sigma, n_tau) || !finite_all(omega, n_omega) ||
      !finite_all(model, n_omega))
    return BSS_E_INVALID_ARG;
  for (int i = 0; i < n_tau; ++i)
    if (!(sigma[i] > 0.0) || tau[i] < 0.0 || tau[i] > beta) return BSS_E_INVALID_ARG;
  for (int j = 0; j < n_omega; ++j)
    if (!(model[j] > 0.0) || (j > 0 && !(omega[j] > omega[j - 1]))) return BSS_E_INVALID_ARG;
  Mem P;
  P.n = n_tau;
  P.M = n_omega;
  std::vector<double> q;
  trapezoid(omega, n_omega, q);
  P.C.resize((size_t)n_tau * n_omega);
  P.d.resize(n_tau);
  P.mu.resize(n_omega);
  for (int i = 0; i < n_tau; ++i) {
    P.d[i] = G[i] / sigma[i];
    for (int j = 0; j < n_omega; ++j) P.C[(size_t)i * n_omega + j] = -kern(tau[i], omega[j], beta) / sigma[i];
  }
  for (int j = 0; j < n_omega; ++j) P.mu[j] = q[j] * model[j];
  P.svd();
  if (P.s < 1) return BSS_E_NUMERICAL;
  std::vector<double> u(P.s, 0.0);
  if (alpha > 0.0) {
    if (!P.solve(alpha, u)) return BSS_E_NUMERICAL;
  } else {
    // historic alpha: chi^2(alpha) = n_tau, chi^2 increasing in alpha
    const double target = n_tau, ln10 = std::log(10.0), lmin = std::log(1e-8), lmax = std::log(1e12);
    auto f = [&](double la, std::vector<double> &uu, double &val) {
      if (!P.solve(std::exp(la), uu)) return false;
      val = P.chi2() - target;
      return true;
    };
    double hi = lmax, lo, flo, fhi;
    std::vector<double> ulo, uhi(P.s, 0.0);
    if (!f(hi, uhi, fhi)) return BSS_E_NUMERICAL;
    if (fhi < 0.0) return BSS_E_NUMERICAL;   // chi^2 < n already at the largest alpha
    ulo = uhi;
    lo = hi - ln10;
    for (;;) {
      if (!f(lo, ulo, flo)) return BSS_E_NUMERICAL;
      if (flo < 0.0) break;
      hi = lo; fhi = flo; uhi = ulo;
      lo -= ln10;
      if (lo < lmin) return BSS_E_NUMERICAL;
    }
    // Illinois regula falsi on [lo, hi], flo < 0 <= fhi
    int side = 0;
    double la = lo;
    u = ulo;
    for (int it = 0; it < 200; ++it) {
      la = (lo * fhi - hi * flo) / (fhi - flo);
      if (!(la > lo && la < hi)) la = 0.5 * (lo + hi);
      u = (la - lo < hi - la) ? ulo : uhi;
      double fm;
      if (!f(la, u, fm)) return BSS_E_NUMERICAL;
      if (std::fabs(fm) <= 1e-12 * target || hi - lo <= 1e-14 * std::max(1.0, std::fabs(la))) break;
      if (fm < 0.0) {
        lo = la; flo = fm; ulo = u;
        if (side == -1) fhi *= 0.5;
        side = -1;
      } else {
        hi = la; fhi = fm; uhi = u;
        if (side == 1) flo *= 0.5;
        side = 1;
      }
    }
    alpha = std::exp(la);
  }
  for (int j = 0; j < n_omega; ++j) A[j] = P.a[j] / q[j];
  if (alpha_out) *alpha_out = alpha;
  if (chi2_out) *chi2_out = P.chi2();
  return BSS_OK;
}

bss_status bss_mem_green(double beta, int32_t n_omega, const double *omega, const double *A, int32_t n_tau,
                         const double *tau, double *G_out) {
  if (!(beta > 0.0) || !std::isfinite(beta) || n_omega < 2 || n_tau < 1 || !omega || !A || !tau || !G_out)
    return BSS_E_INVALID_ARG;
  if (!finite_all(omega, n_omega) || !finite_all(A, n_omega) || !finite_all(tau, n_tau)) return BSS_E_INVALID_ARG;
  for (int j = 1; j < n_omega; ++j)
    if (!(omega[j] > omega[j - 1])) return BSS_E_INVALID_ARG;
  for (int i = 0; i < n_tau; ++i)
    if (tau[i] < 0.0 || tau[i] > beta) return BSS_E_INVALID_ARG;
  std::vector<double> q;
  trapezoid(omega, n_omega, q);
  for (int i = 0; i < n_tau; ++i) {
    double v = 0.0;
    for (int j = 0; j < n_omega; ++j) v += q[j] * kern(tau[i], omega[j], beta) * A[j];
    G_out[i] = -v;
  }
  return BSS_OK;
}

}  // extern "C"
