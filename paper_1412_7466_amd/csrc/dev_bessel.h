// FP64 Bessel and Hankel functions of real positive argument for the device.
//
// Written from the classical methods, no vendor special-function code:
//  * large argument (x >= 20): Hankel's asymptotic expansion (DLMF 10.17.5),
//      H_nu(x) ~ sqrt(2/(pi x)) e^{i(x - nu pi/2 - pi/4)} sum_k i^k a_k(nu) / x^k,
//      a_k(nu) = a_{k-1}(nu) (4 nu^2 - (2k-1)^2) / (8 k),
//    summed until the term drops below 1e-17 (the smallest term is ~e^{-2x});
//  * x < 20: Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1} started
//    far above x and normalised by J_0 + 2 sum J_{2k} = 1 (DLMF 10.12.4), with
//    Neumann's series for Y_0 (DLMF 10.8.2 / A&S 9.1.88)
//      (pi/2) Y_0 = (ln(x/2) + gamma) J_0 - 2 sum_{k>=1} (-1)^k J_{2k} / k,
//    and its derivative for Y_1 = -Y_0':
//      (pi/2) Y_1 = -J_0/x + (ln(x/2) + gamma) J_1 + sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1}) / k.
//  * Hankel functions of higher order by the upward recurrence
//      H_{n+1} = (2n/x) H_n - H_{n-1}, which is stable for H (Y dominates).
#pragma once
#include "dev_common.h"

#define GRT_EULER_GAMMA 0.57721566490153286061
#define GRT_PI 3.14159265358979323846
#define GRT_2_PI 0.63661977236758134308  // 2/pi

// J_0, J_1, Y_0, Y_1 at x > 0.
__host__ __device__ __forceinline__ void bessel01(double x, double& j0, double& j1, double& y0, double& y1) {
  if (x >= 20.0) {
    double ix = 1.0 / x;
    // nu = 0 and nu = 1 together: P + iQ = sum_k i^k a_k / x^k
    double p0 = 1.0, q0 = 0.0, p1 = 1.0, q1 = 0.0;
    double t0 = 1.0, t1 = 1.0;
    for (int k = 1; k < 60; ++k) {
      double o = (2.0 * k - 1.0) * (2.0 * k - 1.0);
      double f = ix / (8.0 * k);
      t0 *= (0.0 - o) * f;
      t1 *= (4.0 - o) * f;
      // i^k: k%4 == 1 -> +i, 2 -> -1, 3 -> -i, 0 -> +1
      switch (k & 3) {
        case 1: q0 += t0; q1 += t1; break;
        case 2: p0 -= t0; p1 -= t1; break;
        case 3: q0 -= t0; q1 -= t1; break;
        default: p0 += t0; p1 += t1; break;
      }
      if (fabs(t0) < 1e-17 && fabs(t1) < 1e-17) break;
    }
    double s, c;
    sincos(x, &s, &c);
    double amp = sqrt(GRT_2_PI * ix);
    // e^{i(x - pi/4)} = ((c + s) + i (s - c)) / sqrt(2)
    const double r2 = 0.70710678118654752440;
    double er = (c + s) * r2, ei = (s - c) * r2;
    // H_0 = amp * e * (p0 + i q0)
    j0 = amp * (er * p0 - ei * q0);
    y0 = amp * (er * q0 + ei * p0);
    // H_1 = amp * e * (-i) * (p1 + i q1) = amp * e * (q1 - i p1)
    j1 = amp * (er * q1 + ei * p1);
    y1 = amp * (ei * q1 - er * p1);
    return;
  }
  // Miller: start at an even order well above x
  int N = ((int)x + 34) & ~1;
  double jp = 0.0, jc = 1e-30;  // J_{N+1}, J_N (unnormalised)
  double seven = 0.0;           // sum_{k>=1} J_{2k}
  double sy0 = 0.0;             // sum_{k>=1} (-1)^k J_{2k} / k
  double sy1 = 0.0;             // sum over odd m of c_m J_m (see header)
  double ix2 = 2.0 / x;
  // J_N itself (N even, N >= 2)
  {
    int k = N >> 1;
    seven += jc;
    sy0 += ((k & 1) ? -jc : jc) / (double)k;
  }
  double jn1 = 0.0;  // will hold J_1
  for (int n = N; n >= 1; --n) {
    double jm = n * ix2 * jc - jp;  // J_{n-1}
    jp = jc;
    jc = jm;
    int m = n - 1;  // order of jc now
    if (m >= 2 && !(m & 1)) {
      int k = m >> 1;
      seven += jc;
      sy0 += ((k & 1) ? -jc : jc) / (double)k;
    } else if (m & 1) {
      int p = m >> 1;  // m = 2p + 1
      double cm = (p == 0) ? -1.0 : (((p & 1) ? 1.0 : -1.0) * (1.0 / p + 1.0 / (p + 1)));
      sy1 += cm * jc;
      if (m == 1) jn1 = jc;
    }
    if (fabs(jc) > 1e250) {  // keep the unnormalised values finite
      const double sc = 1e-250;
      jc *= sc; jp *= sc; seven *= sc; sy0 *= sc; sy1 *= sc; jn1 *= sc;
    }
  }
  double scale = 1.0 / (jc + 2.0 * seven);
  j0 = jc * scale;
  j1 = jn1 * scale;
  sy0 *= scale;
  sy1 *= scale;
  double lg = log(0.5 * x) + GRT_EULER_GAMMA;
  y0 = GRT_2_PI * (lg * j0 - 2.0 * sy0);
  y1 = GRT_2_PI * (-j0 / x + lg * j1 + sy1);
}

__host__ __device__ __forceinline__ void hankel01(double x, cd& h0, cd& h1) {
  double j0, j1, y0, y1;
  bessel01(x, j0, j1, y0, y1);
  h0 = cd{j0, y0};
  h1 = cd{j1, y1};
}

// J_0..J_nmax at x >= 0 into out[0..nmax] (Miller, normalised).
__host__ __device__ inline void bessel_jn_array(double x, int nmax, double* out) {
  if (x < 1e-300) {
    out[0] = 1.0;
    for (int n = 1; n <= nmax; ++n) out[n] = 0.0;
    return;
  }
  int top = nmax > (int)x ? nmax : (int)x;
  int N = (top + 34) & ~1;
  double jp = 0.0, jc = 1e-30, seven = 0.0;
  double ix2 = 2.0 / x;
  if (N <= nmax) out[N] = jc;
  seven += jc;  // N even, >= 2
  for (int n = N; n >= 1; --n) {
    double jm = n * ix2 * jc - jp;
    jp = jc;
    jc = jm;
    int m = n - 1;
    if (m <= nmax) out[m] = jc;
    if (m >= 2 && !(m & 1)) seven += jc;
    if (fabs(jc) > 1e250) {
      const double sc = 1e-250;
      jc *= sc; jp *= sc; seven *= sc;
      int hi = (N < nmax) ? N : nmax;
      for (int q = m; q <= hi; ++q) out[q] *= sc;
    }
  }
  double scale = 1.0 / (jc + 2.0 * seven);
  for (int n = 0; n <= nmax; ++n) out[n] *= scale;
}

// J_{q-1}, J_q, J_{q+1} for any integer q at x >= 0 (Miller, normalised).
__host__ __device__ inline void bessel_j_three(double x, int q, double& jm, double& j0, double& jpl) {
  int aq = q < 0 ? -q : q;
  if (x < 1e-300) {
    jm = (q - 1 == 0) ? 1.0 : 0.0;
    j0 = (q == 0) ? 1.0 : 0.0;
    jpl = (q + 1 == 0) ? 1.0 : 0.0;
    return;
  }
  int top = (aq + 1) > (int)x ? (aq + 1) : (int)x;
  int N = (top + 34) & ~1;
  double jp = 0.0, jc = 1e-30, seven = jc;
  double ix2 = 2.0 / x;
  double v[3] = {0.0, 0.0, 0.0};  // J_{aq-1}, J_aq, J_{aq+1} (unnormalised)
  if (N == aq + 1) v[2] = jc;
  for (int n = N; n >= 1; --n) {
    double jmv = n * ix2 * jc - jp;
    jp = jc;
    jc = jmv;
    int m = n - 1;
    if (m >= 2 && !(m & 1)) seven += jc;
    if (m == aq - 1) v[0] = jc;
    if (m == aq) v[1] = jc;
    if (m == aq + 1) v[2] = jc;
    if (fabs(jc) > 1e250) {
      const double sc = 1e-250;
      jc *= sc; jp *= sc; seven *= sc; v[0] *= sc; v[1] *= sc; v[2] *= sc;
    }
  }
  double scale = 1.0 / (jc + 2.0 * seven);
  double a = v[0] * scale, b = v[1] * scale, c = v[2] * scale;
  if (aq == 0) a = -c;  // J_{-1} = -J_1
  // orders aq-1, aq, aq+1; map to q-1, q, q+1 with J_{-n} = (-1)^n J_n
  if (q >= 0) {
    jm = a; j0 = b; jpl = c;
  } else {
    // q = -aq: J_{q-1} = J_{-(aq+1)} = (-1)^{aq+1} J_{aq+1}, J_q = (-1)^aq J_aq,
    // J_{q+1} = J_{-(aq-1)} = (-1)^{aq-1} J_{aq-1}
    double sg = (aq & 1) ? -1.0 : 1.0;
    jm = -sg * c;
    j0 = sg * b;
    jpl = -sg * a;
  }
}
