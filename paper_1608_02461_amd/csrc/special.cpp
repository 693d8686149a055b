// Host special functions: Bessel/Hankel sequences for the translation
// tables, the near-field polynomial fit, and the two self terms.
#include "special.h"

#include <algorithm>
#include <initializer_list>

namespace hfmm {

void besselj_seq(int nmax, double x, std::vector<double>& J) {
  J.assign(nmax + 1, 0.0);
  for (int n = 0; n <= nmax; ++n) J[n] = (x == 0.0) ? (n == 0 ? 1.0 : 0.0) : std::cyl_bessel_j(double(n), x);
}

void hankel_seq(int nmax, double x, std::vector<std::complex<double>>& H) {
  std::vector<double> J;
  besselj_seq(nmax, x, J);
  H.assign(nmax + 1, 0.0);
  double ym1 = std::cyl_neumann(0.0, x), y = std::cyl_neumann(1.0, x);
  H[0] = {J[0], ym1};
  if (nmax >= 1) H[1] = {J[1], y};
  for (int n = 1; n < nmax; ++n) {  // Y_{n+1} = (2n/x) Y_n - Y_{n-1}, stable upwards
    double yn = 2.0 * n / x * y - ym1;
    ym1 = y;
    y = yn;
    H[n + 1] = {J[n + 1], y};
  }
}

namespace {

// long-double power series of J0(sqrt t) and Yhat(sqrt t), t <= 144
void near_truth(long double t, long double& J, long double& Yh) {
  const long double y = t / 4;
  long double term = 1, H = 0;
  J = 1;
  Yh = 0;
  for (int k = 1; k <= 80; ++k) {
    term *= -y / ((long double)k * k);
    H += 1.0L / k;
    J += term;
    Yh -= H * term;
    if (std::fabs(term) * (1 + H) < 1e-30L) break;
  }
  Yh *= 2.0L / (long double)kPi;
}

template <class F>
double horner(const double* c, int n, double u) {
  F acc = F(c[n - 1]);
  for (int i = n - 2; i >= 0; --i) acc = acc * F(u) + F(c[i]);
  return double(acc);
}

// Chebyshev interpolant of f on [-1,1] with n nodes, returned as monomials in u.
void cheb_to_mono(const std::vector<double>& fvals, int n, double* mono) {
  std::vector<double> c(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += fvals[i] * std::cos(kPi * j * (i + 0.5) / n);
    c[j] = (j == 0 ? 1.0 : 2.0) * s / n;
  }
  // monomial coefficients of T_j by T_{j+1} = 2u T_j - T_{j-1}
  std::vector<double> tm1(n, 0.0), t0(n, 0.0), t1(n, 0.0);
  std::fill(mono, mono + n, 0.0);
  tm1[0] = 1;                 // T_0
  mono[0] += c[0];
  if (n > 1) {
    t0[1] = 1;                // T_1
    mono[1] += c[1];
  }
  for (int j = 2; j < n; ++j) {
    std::fill(t1.begin(), t1.end(), 0.0);
    for (int i = 0; i < n - 1; ++i) t1[i + 1] += 2 * t0[i];
    for (int i = 0; i < n; ++i) t1[i] -= tm1[i];
    for (int i = 0; i < n; ++i) mono[i] += c[j] * t1[i];
    tm1 = t0;
    t0 = t1;
  }
}

}  // namespace

bool fit_near_poly(double tmax, bool fp32, const int* cand, int ncand, int nplain, double tol, NearPoly& out) {
  if (!(tmax > 0) || tmax > 144.0) return false;
  const int nsamp = 4001;
  std::vector<long double> tJ(nsamp), tY(nsamp);
  for (int s = 0; s < nsamp; ++s) near_truth((long double)tmax * s / (nsamp - 1), tJ[s], tY[s]);
  for (int ci = 0; ci < ncand; ++ci) {
    const int n = cand[ci];
    std::vector<double> fJ(n), fY(n);
    for (int i = 0; i < n; ++i) {
      double u = std::cos(kPi * (i + 0.5) / n);
      long double J, Y;
      near_truth((long double)((u + 1) * 0.5 * tmax), J, Y);
      fJ[i] = (double)J;
      fY[i] = (double)Y;
    }
    NearPoly P;
    P.deg = n;
    double mJ[32], mY[32];
    cheb_to_mono(fJ, n, mJ);
    cheb_to_mono(fY, n, mY);
    P.ua = 2.0 / tmax;
    P.ub = -1.0;
    if (ci < nplain) {
      // in t itself: expand sum_k m_k (ua t + ub)^k (exact binomial sums in long double)
      long double a[32] = {0}, b[32] = {0};
      for (int k = 0; k < n; ++k) {
        long double binom = 1, ap = 1;  // C(k, j) ua^j for j = 0 .. k
        for (int j = 0; j <= k; ++j) {
          const long double bp = std::pow((long double)P.ub, (long double)(k - j));
          a[j] += (long double)mJ[k] * binom * ap * bp;
          b[j] += (long double)mY[k] * binom * ap * bp;
          binom = binom * (k - j) / (j + 1);
          ap *= (long double)P.ua;
        }
      }
      for (int j = 0; j < n; ++j) {
        mJ[j] = (double)a[j];
        mY[j] = (double)b[j];
      }
      P.ua = 1.0;
      P.ub = 0.0;
    }
    for (int i = 0; i < n; ++i) {
      P.cJ[i] = P.c1 * mJ[i];
      P.cY[i] = mY[i] + P.c0 * mJ[i];
    }
    double err = 0;
    for (int s = 1; s < nsamp; ++s) {
      double t = tmax * s / (nsamp - 1);
      double u = t * P.ua + P.ub;
      double Jc = fp32 ? horner<float>(P.cJ, n, u) : horner<double>(P.cJ, n, u);
      double Yf = fp32 ? horner<float>(P.cY, n, u) : horner<double>(P.cY, n, u);
      const double J = (double)tJ[s], Yt = (double)tY[s] + P.c0 * J;
      err = std::max(err, std::max(std::fabs(Jc / P.c1 - J), std::fabs(Yf - Yt)));
    }
    P.max_err = err;
    out = P;
    if (err <= tol) return true;
  }
  return false;
}

void gauss_legendre(int n, std::vector<double>& xs, std::vector<double>& ws) {
  // Newton's iteration on P_n from the Chebyshev-like first guess; P_n and
  // P_{n-1} from the three-term recurrence
  xs.assign(n, 0.0);
  ws.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1, p2 = 0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1);
      double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    xs[i] = z;
    ws[i] = 2.0 / ((1 - z * z) * pp * pp);
  }
}

std::complex<double> volume_self_term(double k, double h) {
  // 24-point Gauss-Legendre on [0, pi/4]; the integrand is smooth in theta.
  const int n = 24;
  std::vector<double> xs, ws;
  gauss_legendre(n, xs, ws);
  const double a = 0.0, b = kPi / 4, half = 0.5 * (b - a), mid = 0.5 * (b + a);
  std::complex<double> acc = 0;
  for (int i = 0; i < n; ++i) {
    double th = mid + half * xs[i];
    double R = h / (2 * std::cos(th));
    std::complex<double> H1(std::cyl_bessel_j(1.0, k * R), std::cyl_neumann(1.0, k * R));
    acc += ws[i] * half * (R * H1 / k + std::complex<double>(0, 2.0 / (kPi * k * k)));
  }
  return std::complex<double>(0, 0.25) * 8.0 * acc;
}

std::complex<double> boundary_self_term(double k, double w) {
  const double gam = std::exp(kEulerGamma);
  std::complex<double> v(w, (2.0 / kPi) * w * (std::log(gam * k * w / 4.0) - 1.0));
  return std::complex<double>(0, 0.25) * v;
}

}  // namespace hfmm
