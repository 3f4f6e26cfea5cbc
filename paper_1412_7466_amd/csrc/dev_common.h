// Device-side complex arithmetic and small helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

// Complex FP64, interleaved (re, im) exactly as the coefficient vectors are laid
// out in memory.
struct cd {
  double r, i;
};
// Complex FP32, same layout.
struct cf {
  float r, i;
};

__host__ __device__ __forceinline__ cd cdm(double r, double i) { return cd{r, i}; }
__host__ __device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.r + b.r, a.i + b.i}; }
__host__ __device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.r - b.r, a.i - b.i}; }
__host__ __device__ __forceinline__ cd operator-(cd a) { return cd{-a.r, -a.i}; }
__host__ __device__ __forceinline__ cd operator*(cd a, cd b) {
  return cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
__host__ __device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.r, s * a.i}; }
__host__ __device__ __forceinline__ cd operator*(cd a, double s) { return cd{s * a.r, s * a.i}; }
__host__ __device__ __forceinline__ cd& operator+=(cd& a, cd b) { a.r += b.r; a.i += b.i; return a; }
__host__ __device__ __forceinline__ cd& operator-=(cd& a, cd b) { a.r -= b.r; a.i -= b.i; return a; }
__host__ __device__ __forceinline__ cd conj(cd a) { return cd{a.r, -a.i}; }
__host__ __device__ __forceinline__ double cabs2(cd a) { return a.r * a.r + a.i * a.i; }
__host__ __device__ __forceinline__ cd cdiv(cd a, cd b) {
  double den = b.r * b.r + b.i * b.i;
  return cd{(a.r * b.r + a.i * b.i) / den, (a.i * b.r - a.r * b.i) / den};
}
// acc += a * b
__host__ __device__ __forceinline__ void cmac(cd& acc, cd a, cd b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(a.i, b.r, acc.i);
}
// i * a
__host__ __device__ __forceinline__ cd times_i(cd a) { return cd{-a.i, a.r}; }
// Principal square root; the smaller part from w.i / (2 x the larger) so that a
// nearly real w loses nothing to cancellation.
__host__ __device__ __forceinline__ cd csqrt_principal(cd w) {
  const double a = sqrt(cabs2(w));
  if (a == 0.0) return cd{0.0, 0.0};
  if (w.r >= 0.0) {
    const double re = sqrt(0.5 * (a + w.r));
    return cd{re, w.i / (2.0 * re)};
  }
  const double im = sqrt(0.5 * (a - w.r));
  return cd{fabs(w.i) / (2.0 * im), w.i < 0.0 ? -im : im};
}

__host__ __device__ __forceinline__ cd cexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return cd{c, s};
}

// integer power of a complex number (small non-negative exponents)
__host__ __device__ __forceinline__ cd cpowi(cd a, int n) {
  cd r{1.0, 0.0};
  cd b = a;
  while (n > 0) {
    if (n & 1) r = r * b;
    b = b * b;
    n >>= 1;
  }
  return r;
}
