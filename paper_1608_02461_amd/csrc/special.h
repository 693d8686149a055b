// Cylinder functions for the 2-D Helmholtz kernel G = (i/4) H0^(1)(k r).
//
// Device, full range, FP64 (boundary-matrix assembly and the all-pairs near
// field when the pair distance is not bounded by the tree):
//   x < 4        power series of J0 and Y0 (DLMF 10.2.2, 10.8.2),
//   4 <= x < 20  Miller's backward recurrence for J_n normalised by
//                J0 + 2 sum J_2k = 1, with the Neumann series
//                Y0 = (2/pi)(ln(x/2) + gamma_E) J0 - (4/pi) sum (-1)^k J_2k / k,
//   x >= 20      Hankel's asymptotic expansion (DLMF 10.17.3).
// Host (translation tables): J_n from std::cyl_bessel_j, Y_n by forward
// recurrence from std::cyl_neumann of orders 0 and 1.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

#include "common.h"

namespace hfmm {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kLn2 = 0.69314718055994530942;

// (J0(x), Y0(x)) for x > 0.
__host__ __device__ inline double2 h0_general(double x) {
  double2 r;
  if (x < 4.0) {
    const double y = 0.25 * x * x;
    double t = 1.0, J = 1.0, Yh = 0.0, H = 0.0;
    for (int k = 1; k <= 22; ++k) {
      t *= -y / (double(k) * double(k));
      H += 1.0 / double(k);
      J += t;
      Yh -= H * t;
    }
    r.x = J;
    r.y = (2.0 / kPi) * ((log(0.5 * x) + kEulerGamma) * J + Yh);
  } else if (x < 20.0) {
    int N = (int)x + 30;
    N += N & 1;
    const double inv = 1.0 / x;
    double fp1 = 0.0, f = 1e-30, norm = 0.0, S = 0.0;
    // f holds f_n; walk n = N .. 1 producing f_{n-1}
    for (int n = N; n >= 1; --n) {
      if ((n & 1) == 0) {
        norm += 2.0 * f;
        S += ((n >> 1) & 1 ? -f : f) / double(n >> 1);
      }
      double fm = 2.0 * n * inv * f - fp1;
      fp1 = f;
      f = fm;
    }
    norm += f;
    const double J0 = f / norm;
    r.x = J0;
    r.y = (2.0 / kPi) * ((log(0.5 * x) + kEulerGamma) * J0 - 2.0 * S / norm);
  } else {
    // sum_k i^k a_k / x^k, a_k = -a_{k-1} (2k-1)^2 / (8k)
    double a = 1.0, sr = 1.0, si = 0.0, last = 1.0;
    const double inv = 1.0 / x;
    double xp = 1.0;
    for (int k = 1; k <= 40; ++k) {
      double an = -a * double((2 * k - 1) * (2 * k - 1)) / (8.0 * k);
      xp *= inv;
      double term = an * xp;
      if (fabs(term) > last) break;
      switch (k & 3) {
        case 0: sr += term; break;
        case 1: si += term; break;
        case 2: sr -= term; break;
        default: si -= term; break;
      }
      a = an;
      last = fabs(term);
      if (last < 1e-17) break;
    }
    double s, c;
    sincos(x - 0.25 * kPi, &s, &c);
    const double amp = sqrt(2.0 / (kPi * x));
    r.x = amp * (c * sr - s * si);
    r.y = amp * (s * sr + c * si);
  }
  return r;
}

// (J1(x), Y1(x)) for x > 0, by the same three ranges as h0_general:
//   x < 4        power series (DLMF 10.2.2 and 10.8.1 with n = 1):
//                J1 = (x/2) sum_k t_k,  t_k = (-x^2/4)^k / (k! (k+1)!),
//                Y1 = -2/(pi x) + (2/pi)(ln(x/2) + gamma_E) J1
//                     - (1/pi)(x/2) sum_k (H_k + H_{k+1}) t_k  (H_k harmonic numbers);
//   4 <= x < 20  Miller's backward recurrence (normalised as in h0_general)
//                for J0, J1 and the series obtained by differentiating the
//                Neumann series of Y0 (Y1 = -Y0', J_2k' = (J_{2k-1} - J_{2k+1})/2):
//                Y1 = (2/pi)[(ln(x/2) + gamma_E) J1 - J0/x
//                            + sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1}) / k];
//   x >= 20      Hankel's expansion (DLMF 10.17.3) with nu = 1,
//                a_k = a_{k-1} (4 - (2k-1)^2) / (8k).
__host__ __device__ inline double2 h1_general(double x) {
  double2 r;
  if (x < 4.0) {
    const double y = 0.25 * x * x;
    double t = 1.0, S = 1.0, Hk = 0.0, Hk1 = 1.0, Yh = Hk + Hk1;
    for (int k = 1; k <= 24; ++k) {
      t *= -y / (double(k) * double(k + 1));
      Hk += 1.0 / double(k);
      Hk1 += 1.0 / double(k + 1);
      S += t;
      Yh += (Hk + Hk1) * t;
    }
    const double J1 = 0.5 * x * S;
    r.x = J1;
    r.y = -2.0 / (kPi * x) + (2.0 / kPi) * (log(0.5 * x) + kEulerGamma) * J1 - (0.5 * x / kPi) * Yh;
  } else if (x < 20.0) {
    int N = (int)x + 30;
    N += N & 1;
    const double inv = 1.0 / x;
    double fp1 = 0.0, f = 1e-30, norm = 0.0, S = 0.0, f1 = 0.0;
    // f holds f_n; walk n = N .. 1 producing f_{n-1}
    for (int n = N; n >= 1; --n) {
      if ((n & 1) == 0) {
        norm += 2.0 * f;
      } else {
        // f_n with n = 2k - 1 enters with (-1)^k / k, with n = 2k + 1 (k >= 1) with -(-1)^k / k
        const int ka = (n + 1) >> 1, kb = (n - 1) >> 1;
        S += ((ka & 1) ? -f : f) / double(ka);
        if (kb >= 1) S -= ((kb & 1) ? -f : f) / double(kb);
      }
      if (n == 1) f1 = f;
      double fm = 2.0 * n * inv * f - fp1;
      fp1 = f;
      f = fm;
    }
    norm += f;
    const double J0 = f / norm, J1 = f1 / norm;
    r.x = J1;
    r.y = (2.0 / kPi) * ((log(0.5 * x) + kEulerGamma) * J1 - J0 * inv + S / norm);
  } else {
    double a = 1.0, sr = 1.0, si = 0.0, last = 1.0;
    const double inv = 1.0 / x;
    double xp = 1.0;
    for (int k = 1; k <= 40; ++k) {
      double an = a * double(4 - (2 * k - 1) * (2 * k - 1)) / (8.0 * k);
      xp *= inv;
      double term = an * xp;
      if (fabs(term) > last) break;
      switch (k & 3) {
        case 0: sr += term; break;
        case 1: si += term; break;
        case 2: sr -= term; break;
        default: si -= term; break;
      }
      a = an;
      last = fabs(term);
      if (last < 1e-17) break;
    }
    double s, c;
    sincos(x - 0.75 * kPi, &s, &c);
    const double amp = sqrt(2.0 / (kPi * x));
    r.x = amp * (c * sr - s * si);
    r.y = amp * (s * sr + c * si);
  }
  return r;
}

// Host: n-point Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& xs, std::vector<double>& ws);
// Host: J_n(x) for n = 0..nmax.
void besselj_seq(int nmax, double x, std::vector<double>& J);
// Host: H_n^(1)(x) = J_n + i Y_n for n = 0..nmax, x > 0.
void hankel_seq(int nmax, double x, std::vector<std::complex<double>>& H);

// Near-field polynomial: on t = (k r)^2 in [0, tmax],
//   J0(sqrt t) ~ sum cJ[i] u^i,  Yhat(sqrt t) ~ sum cY[i] u^i,  u = t*ua + ub,
//   Y0 = J0 (c1 log2 t + c0) + Yhat.
// Near-field H0 on t = (k r)^2 in [0, tmax], in the form the pair kernels
// evaluate with u = ua t + ub (u = t for the low-degree, plain forms):
//   Jc(u) = c1 J0(sqrt t)                      (coefficients cJ)
//   Yf(u) = Yhat(sqrt t) + c0 J0(sqrt t)       (coefficients cY)
//   Y0    = Jc log2(t) + Yf,   J0 = Jc / c1,
// where Yhat = Y0 - (2/pi)(ln(sqrt(t)/2) + gamma_E) J0, c1 = ln2/pi and
// c0 = (2/pi)(gamma_E - ln 2).  Folding c0 into Yf and c1 into Jc leaves one
// FMA per pair between the two polynomials, the log2 and the accumulation.
struct NearPoly {
  int deg = 0;  // number of coefficients
  double cJ[32] = {0}, cY[32] = {0};
  double ua = 0, ub = 0;
  // set whether or not a fit is found: the general routine's J0 is scaled by c1 too
  double c1 = 0.69314718055994530942 / 3.14159265358979323846;
  double c0 = (2.0 / 3.14159265358979323846) * (0.57721566490153286061 - 0.69314718055994530942);
  double max_err = 0;  // measured max |error| of J0 and of Yf over the interval
};
// Picks the smallest of the candidate coefficient counts whose error, with
// Horner evaluated in `fp32 ? float : double` on coefficients rounded to it,
// is below tol; returns false if none is (then the general routine must be
// used).  The first `nplain` candidates are polynomials in t itself (ua = 1,
// ub = 0: one FMA less per pair, accurate on short intervals), the others in
// the centred variable u = 2 t / tmax - 1.
bool fit_near_poly(double tmax, bool fp32, const int* cand, int ncand, int nplain, double tol, NearPoly& out);

// Exact integral of G over an h x h cell centred on the node:
// (i/4) int H0(k|x|) dA = (i/4) 8 int_0^{pi/4} [R H1(kR)/k + 2i/(pi k^2)] dtheta, R = h/(2 cos theta).
std::complex<double> volume_self_term(double k, double h);
// The analytic boundary-element diagonal (i/4)[w + i (2/pi) w (ln(gamma k w/4) - 1)].
std::complex<double> boundary_self_term(double k, double w);

}  // namespace hfmm
