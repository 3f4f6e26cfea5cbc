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
    // each series stops at its smallest term (the expansion is asymptotic: near
    // x = 20 its terms turn to grow again around k = 2x before reaching 1e-17)
    double p0 = 1.0, q0 = 0.0, p1 = 1.0, q1 = 0.0;
    double t0 = 1.0, t1 = 1.0;
    bool on0 = true, on1 = true;
    for (int k = 1; k < 60 && (on0 || on1); ++k) {
      double o = (2.0 * k - 1.0) * (2.0 * k - 1.0);
      double f = ix / (8.0 * k);
      const double n0 = t0 * (0.0 - o) * f, n1 = t1 * (4.0 - o) * f;
      on0 = on0 && fabs(n0) < fabs(t0) && fabs(t0) >= 1e-17;
      on1 = on1 && fabs(n1) < fabs(t1) && fabs(t1) >= 1e-17;
      const double a0 = on0 ? n0 : 0.0, a1 = on1 ? n1 : 0.0;
      t0 = n0;
      t1 = n1;
      // i^k: k%4 == 1 -> +i, 2 -> -1, 3 -> -i, 0 -> +1
      switch (k & 3) {
        case 1: q0 += a0; q1 += a1; break;
        case 2: p0 -= a0; p1 -= a1; break;
        case 3: q0 -= a0; q1 -= a1; break;
        default: p0 += a0; p1 += a1; break;
      }
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

// J_0..J_nmax at complex z (absorbing media; |Im z| of order 1 at most) into
// out[0..nmax]: Miller's backward recurrence J_{n-1} = (2n/z) J_n - J_{n+1} from a
// start far above max(nmax, |z|), normalised by J_0 + 2 sum_k J_{2k} = 1 (an identity
// for every complex z).
__host__ __device__ inline void bessel_jn_array_c(cd z, int nmax, cd* out) {
  const double az = sqrt(cabs2(z));
  if (az < 1e-300) {
    out[0] = cd{1.0, 0.0};
    for (int n = 1; n <= nmax; ++n) out[n] = cd{0.0, 0.0};
    return;
  }
  int top = nmax > (int)az ? nmax : (int)az;
  int N = (top + 34) & ~1;
  const cd iz2 = cdiv(cd{2.0, 0.0}, z);
  cd jp{0.0, 0.0}, jc{1e-30, 0.0}, seven{0.0, 0.0};
  if (N <= nmax) out[N] = jc;
  seven += jc;  // N even, >= 2
  for (int n = N; n >= 1; --n) {
    cd jm = (double)n * (iz2 * jc) - jp;
    jp = jc;
    jc = jm;
    int m = n - 1;
    if (m <= nmax) out[m] = jc;
    if (m >= 2 && !(m & 1)) seven += jc;
    if (cabs2(jc) > 1e200) {  // |jc| > 1e100: rescale everything stored so far
      const double sc = 1e-100;
      jc = sc * jc; jp = sc * jp; seven = sc * seven;
      int hi = (N < nmax) ? N : nmax;
      for (int q = m; q <= hi; ++q) out[q] = sc * out[q];
    }
  }
  const cd scale = cdiv(cd{1.0, 0.0}, jc + 2.0 * seven);
  for (int n = 0; n <= nmax; ++n) out[n] = out[n] * scale;
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

// Complex argument (absorbing layers): 0 < |z|, Im z >= 0 and of order one below
// |z| = 20.  J_0, J_1 by Miller's recurrence normalised as for real x, and Y_0, Y_1
// from the same Neumann sums (the identities hold for complex z, with the principal
// ln(z/2)); J and Y grow like e^{Im z} while H = J + iY decays like e^{-Im z}, so H
// keeps about e^{-2 Im z} of the FP64 precision.
__host__ __device__ inline void bessel01_c(cd z, cd& j0, cd& j1, cd& y0, cd& y1) {
  const double az = sqrt(cabs2(z));
  const int N = ((int)az + 34) & ~1;
  const cd iz2 = cdiv(cd{2.0, 0.0}, z);
  cd jp{0.0, 0.0}, jc{1e-30, 0.0}, seven{0.0, 0.0}, sy0{0.0, 0.0}, sy1{0.0, 0.0}, jn1{0.0, 0.0};
  {
    const int k = N >> 1;
    seven += jc;
    sy0 += (((k & 1) ? -1.0 : 1.0) / (double)k) * jc;
  }
  for (int n = N; n >= 1; --n) {
    cd jm = (double)n * (iz2 * jc) - jp;
    jp = jc;
    jc = jm;
    const int m = n - 1;
    if (m >= 2 && !(m & 1)) {
      const int k = m >> 1;
      seven += jc;
      sy0 += (((k & 1) ? -1.0 : 1.0) / (double)k) * jc;
    } else if (m & 1) {
      const int p = m >> 1;
      const double cm = (p == 0) ? -1.0 : (((p & 1) ? 1.0 : -1.0) * (1.0 / p + 1.0 / (p + 1)));
      sy1 += cm * jc;
      if (m == 1) jn1 = jc;
    }
    if (cabs2(jc) > 1e200) {
      const double sc = 1e-100;
      jc = sc * jc; jp = sc * jp; seven = sc * seven; sy0 = sc * sy0; sy1 = sc * sy1;
      jn1 = sc * jn1;
    }
  }
  const cd scale = cdiv(cd{1.0, 0.0}, jc + 2.0 * seven);
  j0 = jc * scale;
  j1 = jn1 * scale;
  sy0 = sy0 * scale;
  sy1 = sy1 * scale;
  const cd lg{log(0.5 * az) + GRT_EULER_GAMMA, atan2(z.i, z.r)};
  y0 = GRT_2_PI * (lg * j0 - 2.0 * sy0);
  y1 = GRT_2_PI * (lg * j1 + sy1 - cdiv(j0, z));
}

// H_0, H_1 at complex z (0 < |z|, Im z >= 0); real z goes to hankel01 above.  For
// |z| >= 20 Hankel's expansion (DLMF 10.17.5, valid for |ph z| < pi) with the
// principal sqrt(2 / (pi z)); below it bessel01_c.
__host__ __device__ inline void hankel01_c(cd z, cd& h0, cd& h1) {
  if (z.i == 0.0 && z.r > 0.0) {
    hankel01(z.r, h0, h1);
    return;
  }
  const double az = sqrt(cabs2(z));
  if (az >= 20.0) {
    const cd iz = cdiv(cd{1.0, 0.0}, z);
    // t_k = i^k a_k(nu) / z^k; each series stops at its smallest term
    cd s0{1.0, 0.0}, s1{1.0, 0.0}, t0{1.0, 0.0}, t1{1.0, 0.0};
    bool on0 = true, on1 = true;
    for (int k = 1; k < 60 && (on0 || on1); ++k) {
      const double o = (2.0 * k - 1.0) * (2.0 * k - 1.0);
      const double f = 1.0 / (8.0 * k);
      const cd n0 = ((0.0 - o) * f) * times_i(t0 * iz);
      const cd n1 = ((4.0 - o) * f) * times_i(t1 * iz);
      on0 = on0 && cabs2(n0) < cabs2(t0) && cabs2(t0) >= 1e-34;
      on1 = on1 && cabs2(n1) < cabs2(t1) && cabs2(t1) >= 1e-34;
      if (on0) s0 += n0;
      if (on1) s1 += n1;
      t0 = n0;
      t1 = n1;
    }
    const cd amp = csqrt_principal(cdiv(cd{GRT_2_PI, 0.0}, z));
    const cd e = exp(-z.i) * cexpi(z.r - 0.25 * GRT_PI);  // e^{i(z - pi/4)}
    const cd ae = amp * e;
    h0 = ae * s0;
    h1 = ae * cd{s1.i, -s1.r};  // e^{-i pi/2} = -i
    return;
  }
  cd j0, j1, y0, y1;
  bessel01_c(z, j0, j1, y0, y1);
  h0 = j0 + times_i(y0);
  h1 = j1 + times_i(y1);
}

// J_{q-1}, J_q, J_{q+1} for any integer q at complex z (Im z of order one; Miller,
// normalised as above).
__host__ __device__ inline void bessel_j_three_c(cd z, int q, cd& jm, cd& j0, cd& jpl) {
  const int aq = q < 0 ? -q : q;
  const double az = sqrt(cabs2(z));
  if (az < 1e-300) {
    jm = cd{(q - 1 == 0) ? 1.0 : 0.0, 0.0};
    j0 = cd{(q == 0) ? 1.0 : 0.0, 0.0};
    jpl = cd{(q + 1 == 0) ? 1.0 : 0.0, 0.0};
    return;
  }
  const int top = (aq + 1) > (int)az ? (aq + 1) : (int)az;
  const int N = (top + 34) & ~1;
  const cd iz2 = cdiv(cd{2.0, 0.0}, z);
  cd jp{0.0, 0.0}, jc{1e-30, 0.0}, seven = jc;
  cd v[3] = {cd{0.0, 0.0}, cd{0.0, 0.0}, cd{0.0, 0.0}};  // J_{aq-1}, J_aq, J_{aq+1}
  if (N == aq + 1) v[2] = jc;
  for (int n = N; n >= 1; --n) {
    cd jmv = (double)n * (iz2 * jc) - jp;
    jp = jc;
    jc = jmv;
    const int m = n - 1;
    if (m >= 2 && !(m & 1)) seven += jc;
    if (m == aq - 1) v[0] = jc;
    if (m == aq) v[1] = jc;
    if (m == aq + 1) v[2] = jc;
    if (cabs2(jc) > 1e200) {
      const double sc = 1e-100;
      jc = sc * jc; jp = sc * jp; seven = sc * seven;
      v[0] = sc * v[0]; v[1] = sc * v[1]; v[2] = sc * v[2];
    }
  }
  const cd scale = cdiv(cd{1.0, 0.0}, jc + 2.0 * seven);
  cd a = v[0] * scale, b = v[1] * scale, c = v[2] * scale;
  if (aq == 0) a = -c;  // J_{-1} = -J_1
  if (q >= 0) {
    jm = a; j0 = b; jpl = c;
  } else {  // J_{-n} = (-1)^n J_n
    const double sg = (aq & 1) ? -1.0 : 1.0;
    jm = (-sg) * c;
    j0 = sg * b;
    jpl = (-sg) * a;
  }
}

// ---------------------------------------------------------------------------
// Fast H_0, H_1 for the apply kernels.
//
// For z >= 1/2 the factor B_nu(t) = H_nu(1/t) e^{-i/t} t^{-1/2}, t = 1/z, is smooth
// and slowly varying on t in [0, 2] (it tends to sqrt(2/pi) e^{-i(nu pi/2 + pi/4)} as
// t -> 0, DLMF 10.17.5).  It is tabulated as piecewise Chebyshev interpolants of
// degree HTAB_DEG on HTAB_NI equal intervals of t, converted to monomials in the
// local variable x in [-1, 1]; the table is built on the device from bessel01 above.
// Then H_nu(z) = B_nu(1/z) e^{iz} z^{-1/2}.  For z < 1/2 the ascending series
// (DLMF 10.2.2, 10.8.1) are summed directly.
// ---------------------------------------------------------------------------
#define HTAB_NI 32
#define HTAB_DEG 8
#define HTAB_TMAX 2.0
#define HTAB_STRIDE (4 * (HTAB_DEG + 1))  // doubles per interval: [coef][B0r, B0i, B1r, B1i]
#define HTAB_SIZE (HTAB_NI * HTAB_STRIDE)

// Coefficients of interval k (out[HTAB_STRIDE]).
__host__ __device__ inline void htab_interval(int k, double* out) {
  const int D = HTAB_DEG, n = D + 1;
  const double w = HTAB_TMAX / HTAB_NI;
  double f[4][HTAB_DEG + 1];
  for (int j = 0; j < n; ++j) {
    double x = cos(GRT_PI * (j + 0.5) / n);
    double t = (k + 0.5) * w + 0.5 * w * x;
    double z = 1.0 / t;
    double j0, j1, y0, y1;
    bessel01(z, j0, j1, y0, y1);
    double s, c;
    sincos(z, &s, &c);
    double sq = sqrt(z);
    // B = H e^{-iz} sqrt(z)
    f[0][j] = sq * (j0 * c + y0 * s);
    f[1][j] = sq * (y0 * c - j0 * s);
    f[2][j] = sq * (j1 * c + y1 * s);
    f[3][j] = sq * (y1 * c - j1 * s);
  }
  for (int fn = 0; fn < 4; ++fn) {
    double ch[HTAB_DEG + 1];
    for (int m = 0; m < n; ++m) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += f[fn][j] * cos(GRT_PI * m * (j + 0.5) / n);
      ch[m] = (m == 0 ? 1.0 : 2.0) * acc / n;
    }
    // Chebyshev -> monomial: T_{m+1} = 2x T_m - T_{m-1}
    double tm1[HTAB_DEG + 1], tm[HTAB_DEG + 1], mono[HTAB_DEG + 1];
    for (int i = 0; i < n; ++i) { tm1[i] = 0.0; tm[i] = 0.0; mono[i] = 0.0; }
    tm1[0] = 1.0;           // T_0
    tm[1] = 1.0;            // T_1
    for (int i = 0; i < n; ++i) mono[i] += ch[0] * tm1[i];
    if (n > 1)
      for (int i = 0; i < n; ++i) mono[i] += ch[1] * tm[i];
    for (int m = 2; m < n; ++m) {
      double nx[HTAB_DEG + 1];
      for (int i = 0; i < n; ++i) nx[i] = (i > 0 ? 2.0 * tm[i - 1] : 0.0) - tm1[i];
      for (int i = 0; i < n; ++i) { tm1[i] = tm[i]; tm[i] = nx[i]; }
      for (int i = 0; i < n; ++i) mono[i] += ch[m] * tm[i];
    }
    for (int i = 0; i < n; ++i) out[4 * i + fn] = mono[i];
  }
}

// Ascending series for z < 1/2 (a dozen terms reach full precision there).
__host__ __device__ __forceinline__ void hankel01_series(double z, cd& h0, cd& h1) {
  double q = 0.25 * z * z;
  double tj0 = 1.0, tj1 = 1.0;  // (-q)^k / (k!)^2, (-q)^k / (k! (k+1)!)
  double j0 = 1.0, j1 = 1.0, s0 = 0.0, s1 = 0.0;
  double hk = 0.0;                                   // harmonic number H_k
  const double g = GRT_EULER_GAMMA;
  s1 = (-g + (1.0 - g));                              // psi(1) + psi(2) at k = 0
  for (int k = 1; k < 12; ++k) {
    tj0 *= -q / ((double)k * k);
    tj1 *= -q / ((double)k * (k + 1));
    j0 += tj0;
    j1 += tj1;
    hk += 1.0 / k;
    s0 += -hk * tj0;                                  // (-1)^{k+1} H_k q^k / (k!)^2
    s1 += (2.0 * (hk - g) + 1.0 / (k + 1)) * tj1;     // (psi(k+1) + psi(k+2)) term
  }
  double hz = 0.5 * z;
  j1 *= hz;
  double lg = log(hz);
  double y0 = GRT_2_PI * ((lg + g) * j0 + s0);
  double y1 = -GRT_2_PI / z + GRT_2_PI * lg * j1 - (hz / GRT_PI) * s1;
  h0 = cd{j0, y0};
  h1 = cd{j1, y1};
}

// H_0, H_1 at z > 0 from the table (tab: HTAB_SIZE doubles, any address space).
template <typename TabPtr>
__host__ __device__ __forceinline__ void hankel01_tab(double z, TabPtr tab, cd& h0, cd& h1) {
  if (z < 1.0 / HTAB_TMAX) {
    hankel01_series(z, h0, h1);
    return;
  }
  double t = 1.0 / z;
  double u = t * (HTAB_NI / HTAB_TMAX);
  int k = (int)u;
  k = k < HTAB_NI - 1 ? k : HTAB_NI - 1;
  double x = 2.0 * (u - k) - 1.0;
  TabPtr c = tab + k * HTAB_STRIDE;
  double a0 = c[4 * HTAB_DEG + 0], a1 = c[4 * HTAB_DEG + 1];
  double a2 = c[4 * HTAB_DEG + 2], a3 = c[4 * HTAB_DEG + 3];
#pragma unroll
  for (int i = HTAB_DEG - 1; i >= 0; --i) {
    a0 = fma(a0, x, c[4 * i + 0]);
    a1 = fma(a1, x, c[4 * i + 1]);
    a2 = fma(a2, x, c[4 * i + 2]);
    a3 = fma(a3, x, c[4 * i + 3]);
  }
  double s, cs;
  sincos(z, &s, &cs);
  double r = sqrt(t);
  double er = cs * r, ei = s * r;
  h0 = cd{er * a0 - ei * a1, er * a1 + ei * a0};
  h1 = cd{er * a2 - ei * a3, er * a3 + ei * a2};
}
