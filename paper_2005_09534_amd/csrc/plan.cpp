// Host FP64 planning math of POLFED: Chebyshev coefficients and the filter
// order from the density of states, and the tridiagonal extremes of the
// bounds Lanczos.
//
// eq. (polyTransf): c_n = sqrt(4 - 3 delta_n0) cos(n arccos sigma); D makes
// P(sigma) = 1.  The order rule (main text, "POLFED algorithm"; Supplement,
// "Convergence of POLFED") asks that the number of eigenvalues of P(H~)
// above p = 0.17 match the number requested: n_P(K) is the integral of a
// Gaussian density of states over the main lobe {x : P_K(x) >= p}; the lobe
// edges come from the closed form of P (with sigma = cos(alpha),
// x = cos(theta), D_K(u) = sin((K+1/2)u)/sin(u/2)):
//     P_K(cos theta) = [D_K(theta-alpha) + D_K(theta+alpha)]
//                      / [D_K(0) + D_K(2 alpha)],
// which follows from 1 + 2 sum_{n<=K} cos(n a) cos(n t) =
// (D_K(t-a) + D_K(t+a))/2.
#include <cmath>
#include <vector>

#include "internal.h"

namespace polfed {

void cheb_coeffs(double sigma, long long K, std::vector<double> &c, double &D, int damping) {
  c.assign((size_t)K + 1, 0.0);
  if (sigma == 0.0) {
    // cos(n pi/2) exactly: 1, 0, -1, 0, ...
    for (long long n = 0; n <= K; ++n) {
      const int r = (int)(n & 3);
      const double cn = (r == 0) ? 1.0 : ((r == 2) ? -1.0 : 0.0);
      c[n] = (n == 0) ? 1.0 : 2.0 * cn;
    }
  } else {
    const double a = std::acos(sigma);
    for (long long n = 0; n <= K; ++n) c[n] = (n == 0 ? 1.0 : 2.0) * std::cos((double)n * a);
  }
  if (damping == POLFED_DAMP_JACKSON) {
    // Jackson damping of the delta expansion: c_n g_n, g_n the Jackson
    // factors for the K + 1 coefficients, D again sum_n c_n T_n(sigma)
    std::vector<double> g;
    jackson((int)(K + 1), g);
    const double a = std::acos(sigma);
    double s = 0.0;
    for (long long n = 0; n <= K; ++n) {
      c[n] *= g[n];
      s += c[n] * std::cos((double)n * a);
    }
    D = s;
    return;
  }
  // D = sum_n c_n T_n(sigma) = 1 + 2 sum_{n>=1} cos^2(n alpha)
  if (sigma == 0.0) {
    D = (double)(K / 2 + 1) + (double)(K / 2);  // 1 + 2 * floor(K/2)
  } else {
    const double a = std::acos(sigma);
    double s = 0.0;
    for (long long n = 0; n <= K; ++n) s += c[n] * std::cos((double)n * a);
    D = s;
  }
}

double dos_gamma(int L, double J1, double J2, double Delta, const double *h) {
  double g2 = L * (J1 * J1 + J2 * J2) * (2.0 + Delta * Delta) / 16.0;
  for (int i = 0; i < L; ++i) g2 += h[i] * h[i] / 4.0;
  return std::sqrt(g2);
}

// Tr H / N in the Sz=0 sector: every pair of distinct sites has
// <S^z_i S^z_j> = -1/(4(L-1)) there, and the field term averages to zero.
double trace_mean(int L, double J1, double J2, double Delta) {
  return -(J1 + J2) * Delta * L / (4.0 * (L - 1));
}

static double dirichlet(double u, long long K) {
  const double sh = std::sin(0.5 * u);
  if (std::fabs(sh) < 1e-12) return 2.0 * (double)K + 1.0;
  return std::sin(((double)K + 0.5) * u) / sh;
}

static double P_theta(double theta, double alpha, long long K) {
  const double num = dirichlet(theta - alpha, K) + dirichlet(theta + alpha, K);
  const double den = dirichlet(0.0, K) + dirichlet(2.0 * alpha, K);
  return num / den;
}

// The Jackson-damped filter in closed form.  The Jackson factors of M
// coefficients are the autocorrelation of a_v = sin(beta (v+1)), beta =
// pi/(M+1), so 1 + 2 sum_{n>=1} g_n cos(n phi) = |A(phi)|^2 / sum a_v^2 with
// A(phi) = sum_v a_v e^{i v phi}; summing the two geometric series,
// |A(phi)| = |E_M(phi + beta) + E_M(phi - beta)| / 2 with E_M(u) =
// sin(M u/2)/sin(u/2).  As for the undamped filter,
//     P^J_K(cos theta) = [F(theta-alpha) + F(theta+alpha)] / [F(0) + F(2 alpha)],
// F(phi) = (E_M(phi+beta) + E_M(phi-beta))^2, M = K + 1.
static double dirichlet_m(double u, long long M) {
  const double sh = std::sin(0.5 * u);
  if (std::fabs(sh) < 1e-12) return (double)M * std::cos(0.5 * (double)M * u) / std::cos(0.5 * u);
  return std::sin(0.5 * (double)M * u) / sh;
}

static double jackson_F(double phi, long long M) {
  const double beta = M_PI / ((double)M + 1.0);
  const double v = dirichlet_m(phi + beta, M) + dirichlet_m(phi - beta, M);
  return v * v;
}

static double P_theta_jackson(double theta, double alpha, long long K) {
  const long long M = K + 1;
  return (jackson_F(theta - alpha, M) + jackson_F(theta + alpha, M)) /
         (jackson_F(0.0, M) + jackson_F(2.0 * alpha, M));
}

static double P_theta_of(int damping, double theta, double alpha, long long K) {
  return damping == POLFED_DAMP_JACKSON ? P_theta_jackson(theta, alpha, K)
                                        : P_theta(theta, alpha, K);
}

// Bisection on [alpha, t_out] for the crossing P = p; P(alpha) = 1 >= p.
static double lobe_edge(double alpha, double t_out, long long K, double p, int damping) {
  double t_in = alpha;
  if (P_theta_of(damping, t_out, alpha, K) >= p) return t_out;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (t_in + t_out);
    if (mid == t_in || mid == t_out) break;
    if (P_theta_of(damping, mid, alpha, K) >= p)
      t_in = mid;
    else
      t_out = mid;
  }
  return t_in;
}

// Edges (x_lo, x_hi) of the main lobe {P_K >= p} around sigma: searched
// within the first zero of the undamped kernel (2 pi/(2K+1) from alpha) or,
// damped, within twice the damped kernel's first zero (3 pi/(K+2)); beyond
// those the side lobes stay below p.
static void lobe(long long K, double sigma, double p, double &x_lo, double &x_hi, int damping) {
  const double alpha = std::acos(sigma);
  const double w = damping == POLFED_DAMP_JACKSON ? 6.0 * M_PI / ((double)K + 2.0)
                                                  : 2.0 * M_PI / (2.0 * (double)K + 1.0);
  const double th_r = lobe_edge(alpha, std::min(alpha + w, M_PI), K, p, damping);
  const double th_l = lobe_edge(alpha, std::max(alpha - w, 0.0), K, p, damping);
  x_lo = std::cos(th_r);
  x_hi = std::cos(th_l);
}

static double n_in_window(long long K, double sigma, double p, long long N, double Ebar,
                          double Gamma, double E0w, double E1w, int damping) {
  double x_lo, x_hi;
  lobe(K, sigma, p, x_lo, x_hi, damping);
  const double Elo = 0.5 * (x_lo * (E1w - E0w) + (E1w + E0w));
  const double Ehi = 0.5 * (x_hi * (E1w - E0w) + (E1w + E0w));
  const double s = std::sqrt(2.0) * Gamma;
  return 0.5 * (double)N * (std::erf((Ehi - Ebar) / s) - std::erf((Elo - Ebar) / s));
}

// K = max{K : f(K) >= nwin} by doubling and bisection (f falls with K).
template <class F>
static long long order_rule(F &&f, int nwin) {
  const long long Kmax = 1LL << 26;
  if (f(1) < nwin) return 1;
  long long lo = 1, hi = 2;
  while (hi <= Kmax && f(hi) >= nwin) {
    lo = hi;
    hi *= 2;
  }
  if (hi > Kmax) return Kmax;
  while (hi - lo > 1) {
    const long long mid = (lo + hi) / 2;
    if (f(mid) >= nwin)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

long long choose_order(long long N, double Ebar, double Gamma, double E0w, double E1w,
                       double sigma, int nwin, double p, double *rho, int damping) {
  if (rho) {
    const double E = 0.5 * (sigma * (E1w - E0w) + (E1w + E0w));
    *rho = (double)N * (E1w - E0w) / (2.0 * std::sqrt(2.0 * M_PI) * Gamma) *
           std::exp(-(E - Ebar) * (E - Ebar) / (2.0 * Gamma * Gamma));
  }
  return order_rule(
      [&](long long K) { return n_in_window(K, sigma, p, N, Ebar, Gamma, E0w, E1w, damping); },
      nwin);
}

// ---- density of states by the kernel polynomial method --------------------
//
// With Chebyshev moments mu_n = Tr T_n(H~) / N of H~ (estimated from random
// vectors, Silver et al.), the Jackson-damped density is
//   rho(x) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (pi sqrt(1 - x^2)),
//   g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))] / (M+1)
// (Weisse et al., Rev. Mod. Phys. 78, 275 (2006)), and with x = cos(theta)
// the number of states in [x_lo, x_hi] integrates in closed form:
//   N / pi [g_0 mu_0 (t_lo - t_hi) + 2 sum g_n mu_n (sin n t_lo - sin n t_hi)/n].

void jackson(int M, std::vector<double> &g) {
  g.resize(M);
  const double a = M_PI / (M + 1);
  for (int n = 0; n < M; ++n)
    g[n] = ((M - n + 1) * std::cos(a * n) + std::sin(a * n) / std::tan(a)) / (M + 1);
}

double kpm_count(const std::vector<double> &mu, long long N, double x_lo, double x_hi) {
  const int M = (int)mu.size();
  std::vector<double> g;
  jackson(M, g);
  const double tl = std::acos(std::max(-1.0, std::min(1.0, x_lo)));
  const double th = std::acos(std::max(-1.0, std::min(1.0, x_hi)));
  double s = g[0] * mu[0] * (tl - th);
  for (int n = 1; n < M; ++n) s += 2.0 * g[n] * mu[n] * (std::sin(n * tl) - std::sin(n * th)) / n;
  return (double)N * s / M_PI;
}

double kpm_density(const std::vector<double> &mu, double x) {
  const int M = (int)mu.size();
  std::vector<double> g;
  jackson(M, g);
  const double t = std::acos(std::max(-1.0, std::min(1.0, x)));
  double s = g[0] * mu[0];
  for (int n = 1; n < M; ++n) s += 2.0 * g[n] * mu[n] * std::cos(n * t);
  return s / (M_PI * std::sqrt(std::max(1e-300, 1.0 - x * x)));
}

long long choose_order_kpm(const std::vector<double> &mu, long long N, double sigma, int nwin,
                           double p, int damping) {
  return order_rule(
      [&](long long K) {
        double x_lo, x_hi;
        lobe(K, sigma, p, x_lo, x_hi, damping);
        return kpm_count(mu, N, x_lo, x_hi);
      },
      nwin);
}

// The smallest window count N >= nwin whose order K(N) = choose_order(N)
// does not exceed K_cap (K_cap <= 0: no cap, N = nwin).  K(N) falls as N
// grows (a wider window needs a shorter filter: N_ev -> alpha N_ev gives
// K -> K / alpha at about the same total filter work; Supplement,
// "Benchmark for disorder spin chains"), so N is found by doubling and
// bisection; it is at most the sector size.  Writes that order to *K.
template <class O>
static int capped_window_by(O &&order, long long N, int nwin, long long K_cap, long long *K) {
  long long k = order(nwin);
  if (K_cap <= 0 || k <= K_cap || nwin >= N) {
    *K = k;
    return nwin;
  }
  long long lo = nwin, hi = nwin;  // order(lo) > K_cap
  for (;;) {
    hi = std::min<long long>(N, 2 * hi);
    if (order(hi) <= K_cap || hi == N) break;
    lo = hi;
  }
  while (hi - lo > 1) {
    const long long mid = (lo + hi) / 2;
    if (order(mid) <= K_cap)
      hi = mid;
    else
      lo = mid;
  }
  *K = order(hi);
  return (int)hi;
}

int capped_window(long long N, double Ebar, double Gamma, double E0w, double E1w, double sigma,
                  int nwin, double p, long long K_cap, long long *K, int damping) {
  return capped_window_by(
      [&](long long w) {
        return choose_order(N, Ebar, Gamma, E0w, E1w, sigma, (int)w, p, nullptr, damping);
      },
      N, nwin, K_cap, K);
}

int capped_window_kpm(const std::vector<double> &mu, long long N, double sigma, int nwin,
                      double p, long long K_cap, long long *K, int damping) {
  return capped_window_by(
      [&](long long w) { return choose_order_kpm(mu, N, sigma, (int)w, p, damping); }, N, nwin,
      K_cap, K);
}

// ---- tridiagonal extremes (bounds Lanczos) --------------------------------

// number of eigenvalues < x of the tridiagonal (a[0..m), b[1..m) off-diag)
static int sturm_count(const std::vector<double> &a, const std::vector<double> &b, double x) {
  int cnt = 0;
  double q = 1.0;
  const size_t m = a.size();
  for (size_t i = 0; i < m; ++i) {
    const double bb = (i == 0) ? 0.0 : b[i] * b[i];
    q = a[i] - x - ((i == 0) ? 0.0 : bb / q);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// last component of the unit eigenvector for eigenvalue lam, by two steps
// of inverse iteration on the definite matrix s (T - mu I), mu just outside
// the spectrum (below for the lowest, above for the highest eigenvalue), so
// that the LDL^T solve needs no pivoting.
static double last_component(const std::vector<double> &a, const std::vector<double> &b,
                             double mu, double sgn) {
  const size_t m = a.size();
  std::vector<double> d(m), l(m), y(m, 1.0);
  // M = sgn (T - mu I), positive definite
  for (int it = 0; it < 3; ++it) {
    for (size_t i = 0; i < m; ++i) {
      const double di = sgn * (a[i] - mu);
      if (i == 0) {
        d[i] = di;
      } else {
        const double off = sgn * b[i];
        l[i] = off / d[i - 1];
        d[i] = di - l[i] * off;
      }
      if (d[i] == 0.0) d[i] = 1e-300;
    }
    for (size_t i = 1; i < m; ++i) y[i] -= l[i] * y[i - 1];
    for (size_t i = 0; i < m; ++i) y[i] /= d[i];
    for (size_t i = m - 1; i-- > 0;) y[i] -= l[i + 1] * y[i + 1];
    double nrm = 0.0;
    for (size_t i = 0; i < m; ++i) nrm += y[i] * y[i];
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < m; ++i) y[i] /= nrm;
  }
  return y[m - 1];
}

void tridiag_extremes(const std::vector<double> &a, const std::vector<double> &b, double &lo,
                      double &hi, double &ylo_last, double &yhi_last) {
  const size_t m = a.size();
  double gl = a[0], gu = a[0];
  for (size_t i = 0; i < m; ++i) {
    const double r = ((i > 0) ? std::fabs(b[i]) : 0.0) + ((i + 1 < m) ? std::fabs(b[i + 1]) : 0.0);
    gl = std::min(gl, a[i] - r);
    gu = std::max(gu, a[i] + r);
  }
  const double span = std::max(gu - gl, 1e-300);
  auto bisect = [&](int k) {  // k-th smallest eigenvalue (0-based)
    double l = gl - 1e-12 * span, u = gu + 1e-12 * span;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + u);
      if (mid == l || mid == u) break;
      if (sturm_count(a, b, mid) > k)
        u = mid;
      else
        l = mid;
    }
    return 0.5 * (l + u);
  };
  lo = bisect(0);
  hi = bisect((int)m - 1);
  const double eps = 1e-13 * span;
  ylo_last = last_component(a, b, lo - eps, 1.0);
  yhi_last = last_component(a, b, hi + eps, -1.0);
}

}  // namespace polfed
