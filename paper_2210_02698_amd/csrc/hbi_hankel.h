// FP64 Hankel functions H0^(1), H1^(1) of real positive argument, written
// from the classical expansions (no vendor math code):
//   x < 3      ascending power series of J0, J1, Y0, Y1;
//   3 <= x < 20 Miller's backward recurrence for J_k, normalised by
//              J0 + 2 sum J_2k = 1, with Y0 and Y1 from the Neumann series
//              Y0 = (2/pi)(ln(x/2)+gamma) J0 - (4/pi) sum (-1)^k J_2k / k
//              Y1 = -(2/(pi x)) J0 + (2/pi)(ln(x/2)+gamma) J1
//                   + (2/pi) sum (-1)^k (J_{2k-1} - J_{2k+1}) / k
//              (the second is minus the derivative of the first);
//   x >= 20    Hankel's asymptotic expansion
//              H_nu(x) ~ sqrt(2/(pi x)) e^{i(x - nu pi/2 - pi/4)}
//                        sum_k i^k a_k(nu) / x^k,
//              a_k = a_{k-1} (4 nu^2 - (2k-1)^2) / (8k), truncated at the
//              smallest term.
// Relative accuracy of the complex values is about 2e-15 on (0, 3000].
#pragma once
#include <math.h>

#ifndef HBI_HD
#define HBI_HD __host__ __device__
#endif

namespace hbi {

constexpr double kPi = 3.14159265358979323846;
constexpr double kGamma = 0.57721566490153286061;
constexpr double kInvSqrt2 = 0.70710678118654752440;

struct Hankel01 { double j0, y0, j1, y1; };

HBI_HD inline Hankel01 hankel01_series(double x) {
  const double q = 0.25 * x * x;
  double t0 = 1.0, t1 = 1.0, j0 = 1.0, j1 = 1.0, s0 = 0.0;
  double H = 0.0;
  // Y1 series coefficient psi(k+1) + psi(k+2) with psi(k+1) = H_k - gamma.
  double s1 = 1.0 - 2.0 * kGamma;
  for (int k = 1; k < 40; ++k) {
    t0 *= -q / double(k * k);
    t1 *= -q / double(k * (k + 1));
    H += 1.0 / k;
    j0 += t0;
    j1 += t1;
    s0 -= t0 * H;
    s1 += t1 * (2.0 * H - 2.0 * kGamma + 1.0 / (k + 1));
    if (fabs(t0) < 1e-18 && fabs(t1) < 1e-18) break;
  }
  const double half = 0.5 * x;
  j1 *= half;
  const double lg = log(half);
  Hankel01 r;
  r.j0 = j0;
  r.j1 = j1;
  r.y0 = (2.0 / kPi) * ((lg + kGamma) * j0 + s0);
  r.y1 = -2.0 / (kPi * x) + (2.0 / kPi) * lg * j1 - (1.0 / kPi) * half * s1;
  return r;
}

HBI_HD inline Hankel01 hankel01_miller(double x) {
  // even start index comfortably above x: x + 12 + 6 x^(1/3), with x^(1/3)
  // bounded by its tangent at x = 3 (so the start is never lower)
  int N = (int)(x + 12.0 + 6.0 * (1.4422495703074083 + 0.16025 * (x - 3.0)));
  N = (N / 2) * 2 + 2;
  const double inv = 2.0 / x;
  double jp1 = 0.0, jk = 1e-30;        // J_{k+1}, J_k (unnormalised), k = N
  double norm = 0.0, sy0 = 0.0, sy1 = 0.0, j1 = 0.0;
  // pairs k = 2m (even), 2m - 1 (odd), m = N/2 .. 1; one reciprocal per pair
  int m = N / 2;
  double sg = (m & 1) ? -1.0 : 1.0;    // (-1)^m
  double rm = 1.0 / m;
  for (; m >= 1; --m) {
    // J_{2m}: normalisation and Y0 sums
    norm += 2.0 * jk;
    sy0 += sg * jk * rm;
    double jm1 = (2 * m) * inv * jk - jp1;   // J_{2m-1}
    jp1 = jk;
    jk = jm1;
    // J_{2m-1} enters Y1 as (-1)^m / m and, for m >= 2, as (-1)^m / (m - 1)
    const double rm1 = m >= 2 ? 1.0 / (m - 1) : 0.0;
    sy1 += sg * jk * (rm + rm1);
    if (m == 1) j1 = jk;
    jm1 = (2 * m - 1) * inv * jk - jp1;       // J_{2m-2}
    jp1 = jk;
    jk = jm1;
    if (fabs(jk) > 1e250) {
      jk *= 1e-250; jp1 *= 1e-250; norm *= 1e-250; sy0 *= 1e-250;
      sy1 *= 1e-250; j1 *= 1e-250;
    }
    sg = -sg;
    rm = rm1;
  }
  norm += jk;                      // J_0
  const double s = 1.0 / norm;
  const double J0 = jk * s, J1 = j1 * s;
  const double lg = log(0.5 * x) + kGamma;
  Hankel01 r;
  r.j0 = J0;
  r.j1 = J1;
  r.y0 = (2.0 / kPi) * lg * J0 - (4.0 / kPi) * sy0 * s;
  r.y1 = -(2.0 / (kPi * x)) * J0 + (2.0 / kPi) * lg * J1 + (2.0 / kPi) * sy1 * s;
  return r;
}

HBI_HD inline Hankel01 hankel01_asym(double x) {
  double sn, cs;
  sincos(x, &sn, &cs);
  // e^{i(x - pi/4)}
  const double er = (cs + sn) * kInvSqrt2, ei = (sn - cs) * kInvSqrt2;
  const double amp = sqrt(2.0 / (kPi * x));
  double out[4];
  for (int nu = 0; nu < 2; ++nu) {
    const double mu = 4.0 * nu * nu;
    double a = 1.0, sr = 1.0, si = 0.0, prev = 1e300;
    for (int k = 1; k < 60; ++k) {
      a *= (mu - double((2 * k - 1) * (2 * k - 1))) / (8.0 * k * x);
      const double aa = fabs(a);
      if (aa > prev || aa < 1e-17) break;
      prev = aa;
      switch (k & 3) {
        case 0: sr += a; break;
        case 1: si += a; break;
        case 2: sr -= a; break;
        default: si -= a; break;
      }
    }
    // phase factor e^{i(x - pi/4)} (-i)^nu
    const double pr = nu ? ei : er, pi_ = nu ? -er : ei;
    out[2 * nu] = amp * (sr * pr - si * pi_);      // J_nu
    out[2 * nu + 1] = amp * (sr * pi_ + si * pr);  // Y_nu
  }
  Hankel01 r;
  r.j0 = out[0]; r.y0 = out[1]; r.j1 = out[2]; r.y1 = out[3];
  return r;
}

HBI_HD inline Hankel01 hankel01(double x) {
  if (x < 3.0) return hankel01_series(x);
  if (x < 20.0) return hankel01_miller(x);
  return hankel01_asym(x);
}

}  // namespace hbi
