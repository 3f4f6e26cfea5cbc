// The field at arbitrary points from the discrete representation (paper sec. 2
// problem statement, sec. 3 eqs. repre1-repre3, sec. 5 eq. repre3_mod, sec. 4.1 for
// the inside of the disks).
//
// One lane per point.  By region:
//   y > y0        sum_n c_n e^{i kappa_n x + i k_{1,n} (y - y0)} + incident wave
//   h < y <= y0   S_{k1} sigma_1 + D_{k1} mu_1 (three copies of Gamma_1, node sums)
//                 + sum_q a1_q J_q(k1 |x - c1|) e^{iq theta} + incident wave
//   |y| <= h      the middle layer: S_{k2}, D_{k2} on both interfaces, the middle J
//                 expansion, and the outgoing multipoles of every disk and of its
//                 two near copies; inside a disk (or a copy, phase alpha^l) the
//                 interior expansion sum_n gamma_n J_n(k_p r) e^{in theta}
//   -y0 <= y < -h S_{k3} sigma_2 + D_{k3} mu_2 + sum_q a3_q J_q(k3 |x - c3|) e^{iq theta}
//   y < -y0       sum_n d_n e^{i kappa_n x - i k_{3,n} (y + y0)}
// The layer potentials are the trapezoid sums over the interface nodes the method
// solves with: exact to rounding a few node spacings from an interface, not on it.
// gamma_n = (a_n J_n(k2 R) + beta_n H_n(k2 R)) / J_n(k_p R) with a = T beta +
// B_phys A^+ (f - C beta) the field arriving at the disk.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

struct FieldIn {
  DevGeom g;
  const cd* alpha;   // [n_alpha] unscaled layer unknowns
  const cd* beta;    // [M][nb]
  const cd* gam;     // [M][nb] interior coefficients
  const double *cx, *cy, *rad, *kp;
  const double* htab;
  double k1cos;      // k1 cos(phi)
};

__device__ cd sqrt_branch(double v) {
  return v >= 0 ? cd{sqrt(v), 0.0} : cd{0.0, sqrt(-v)};
}

__device__ cd cexp_c(cd z) {  // e^z
  const double m = exp(z.r);
  double s, c;
  sincos(z.i, &s, &c);
  return cd{m * c, m * s};
}

// Three copies of S_k sigma + D_k mu from the line y = ys (node sums, weight d/N).
__device__ cd line_field(const FieldIn& in, double k, double ys, const cd* sig, const cd* mu,
                         double x, double y) {
  const DevGeom& g = in.g;
  const cd wl[3] = {g.alpha_inv, cd{1.0, 0.0}, g.alpha};
  cd acc{0, 0};
  for (int l = -1; l <= 1; ++l) {
    cd s{0, 0};
    for (int i = 0; i < g.N; ++i) {
      const double xs = -0.5 * g.d + (i + 0.5) * g.hs + l * g.d;
      const double Rx = x - xs, Ry = y - ys;
      const double r = sqrt(Rx * Rx + Ry * Ry);
      if (r < 1e-300) continue;
      cd h0, h1;
      hankel01_tab(k * r, in.htab, h0, h1);
      // (i/4) H0 sigma + (i k / 4) H1 (Ry / r) mu
      const cd a = times_i(0.25 * h0);
      const cd b = times_i((0.25 * k * Ry / r) * h1);
      s += a * sig[i] + b * mu[i];
    }
    s = s * wl[l + 1];
    acc += s;
  }
  return g.hs * acc;
}

// sum_{q=-Q..Q} a[Q+q] J_q(k r) e^{iq theta} about (0, yc): Miller's backward
// recurrence accumulated on the fly (J_{-q} = (-1)^q J_q), normalised by
// J_0 + 2 sum J_{2k} = 1 at the end.
__device__ cd jexp(const cd* a, int Q, double k, double yc, double x, double y) {
  const double vx = x, vy = y - yc;
  const double r = sqrt(vx * vx + vy * vy);
  if (r < 1e-300) return a[Q];
  const double z = k * r;
  const cd e{vx / r, vy / r};
  if (z < 1e-10) {  // J_0 = 1, J_{+-1} = +-z/2, higher orders below rounding
    const double h = Q >= 1 ? 0.5 * z : 0.0;
    return Q >= 1 ? a[Q] + h * (a[Q + 1] * e - a[Q - 1] * conj(e)) : a[Q];
  }
  const cd einv = conj(e);
  int top = Q > (int)z ? Q : (int)z;
  const int N = (top + 34) & ~1;
  double jp = 0.0, jc = 1e-30, seven = jc;
  const double ix2 = 2.0 / z;
  cd eq = cpowi(e, Q);   // e^{i q theta} for the current q <= Q, stepped down
  cd S{0, 0};
  for (int n = N; n >= 1; --n) {
    const double jm = n * ix2 * jc - jp;
    jp = jc;
    jc = jm;
    const int m = n - 1;
    if (m >= 2 && !(m & 1)) seven += jc;
    if (m <= Q) {
      cd cm;
      if (m == 0) {
        cm = a[Q];
      } else {
        const double sg = (m & 1) ? -1.0 : 1.0;
        cm = a[Q + m] * eq + (sg * a[Q - m]) * conj(eq);
      }
      S += jc * cm;
      eq = eq * einv;
    }
    if (fabs(jc) > 1e250) {
      const double sc = 1e-250;
      jc *= sc;
      jp *= sc;
      seven *= sc;
      S = sc * S;
    }
  }
  return (1.0 / (jc + 2.0 * seven)) * S;
}

__global__ void __launch_bounds__(64) field_kernel(FieldIn in, int n_pts, const double* xy, cd* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  const DevGeom& g = in.g;
  // the representation holds in the unit cell |x| <= d/2; elsewhere the field
  // follows from quasi-periodicity, u(x + l d) = alpha^l u(x)
  const double x0 = xy[2 * p], y = xy[2 * p + 1];
  const double cellf = floor(x0 / g.d + 0.5);
  const double x = x0 - cellf * g.d;
  const int cell = (int)cellf;
  const cd cell_phase = cell >= 0 ? cpowi(g.alpha, cell) : cpowi(g.alpha_inv, -cell);
  const cd* mu1 = in.alpha + g.col_off[CB_MU1];
  const cd* sig1 = in.alpha + g.col_off[CB_SIG1];
  const cd* mu2 = in.alpha + g.col_off[CB_MU2];
  const cd* sig2 = in.alpha + g.col_off[CB_SIG2];
  const cd uinc = cexpi(g.kappa * x - in.k1cos * y);
  cd u{0, 0};
  if (y > g.y0 || y < -g.y0) {
    const bool top = y > g.y0;
    const cd* coef = in.alpha + g.col_off[top ? CB_C : CB_D];
    const double kk = top ? g.k[0] : g.k[2];
    for (int i = 0; i < g.Nrb; ++i) {
      const double kap = g.kappa + 2.0 * M_PI * (g.n_rb_lo + i) / g.d;
      const cd kn = sqrt_branch(kk * kk - kap * kap);
      const double dy = top ? (y - g.y0) : -(y + g.y0);
      // e^{i kap x + i kn dy}
      const cd ph = cexp_c(cd{-kn.i * dy, kap * x + kn.r * dy});
      u += coef[i] * ph;
    }
    if (top) u += uinc;
  } else if (y > g.h) {
    u = line_field(in, g.k[0], g.h, sig1, mu1, x, y) +
        jexp(in.alpha + g.col_off[CB_A1], g.Q[0], g.k[0], g.jcy[0], x, y) + uinc;
  } else if (y < -g.h) {
    u = line_field(in, g.k[2], -g.h, sig2, mu2, x, y) +
        jexp(in.alpha + g.col_off[CB_A3], g.Q[2], g.k[2], g.jcy[2], x, y);
  } else {
    const int P = g.P, nb = 2 * P + 1;
    const cd wl[3] = {g.alpha_inv, cd{1.0, 0.0}, g.alpha};
    // inside a disk or one of its near copies?
    int im = -1, il = 0;
    for (int m = 0; m < g.M && im < 0; ++m)
      for (int l = -1; l <= 1; ++l) {
        const double vx = x - in.cx[m] - l * g.d, vy = y - in.cy[m];
        if (vx * vx + vy * vy < in.rad[m] * in.rad[m]) {
          im = m;
          il = l;
          break;
        }
      }
    if (im >= 0) {
      const double vx = x - in.cx[im] - il * g.d, vy = y - in.cy[im];
      const double r = sqrt(vx * vx + vy * vy);
      double jn[41];
      bessel_jn_array(in.kp[im] * r, P, jn);
      const cd e = r > 1e-300 ? cd{vx / r, vy / r} : cd{1.0, 0.0};
      const cd* gm = in.gam + (size_t)im * nb;
      cd s = gm[P] * jn[0];
      cd ep = e;
      for (int n = 1; n <= P; ++n) {
        const double sg = (n & 1) ? -1.0 : 1.0;
        s += jn[n] * (gm[P + n] * ep + (sg * gm[P - n]) * conj(ep));
        ep = ep * e;
      }
      u = wl[il + 1] * s;
    } else {
      u = line_field(in, g.k[1], g.h, sig1, mu1, x, y) +
          line_field(in, g.k[1], -g.h, sig2, mu2, x, y) +
          jexp(in.alpha + g.col_off[CB_A2], g.Q[1], g.k[1], g.jcy[1], x, y);
      const double k2 = g.k[1];
      for (int m = 0; m < g.M; ++m) {
        const cd* b = in.beta + (size_t)m * nb;
        for (int l = -1; l <= 1; ++l) {
          const double vx = x - in.cx[m] - l * g.d, vy = y - in.cy[m];
          const double r = sqrt(vx * vx + vy * vy);
          const double z = k2 * r;
          cd hm, hc;   // H_{n-1}, H_n
          hankel01_tab(z, in.htab, hm, hc);
          const cd e{vx / r, vy / r};
          cd s = b[P] * hm;   // n = 0
          cd ep = e;
          const double i2z = 2.0 / z;
          for (int n = 1; n <= P; ++n) {
            // hc = H_n here
            const double sg = (n & 1) ? -1.0 : 1.0;
            s += hc * (b[P + n] * ep + (sg * b[P - n]) * conj(ep));
            const cd hn = (n * i2z) * hc - hm;
            hm = hc;
            hc = hn;
            ep = ep * e;
          }
          u += wl[l + 1] * s;
        }
      }
    }
  }
  out[p] = cell_phase * u;
}

// gamma_m[n] = (a_n J_n(k2 R) + beta_n H_n(k2 R)) / J_n(k_p R), one lane per disk.
__global__ void __launch_bounds__(64) interior_kernel(int M, int P, double k2, const double* rad,
                                                      const double* kp, const cd* a, const cd* beta,
                                                      cd* gam) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int nb = 2 * P + 1;
  const double R = rad[m];
  double j2[41], jp[41];
  bessel_jn_array(k2 * R, P, j2);
  bessel_jn_array(kp[m] * R, P, jp);
  cd hm, hc;
  hankel01(k2 * R, hm, hc);
  cd h[41];
  h[0] = hm;
  if (P >= 1) h[1] = hc;
  for (int n = 1; n < P; ++n) h[n + 1] = (2.0 * n / (k2 * R)) * h[n] - h[n - 1];
  for (int n = -P; n <= P; ++n) {
    const int an = n < 0 ? -n : n;
    const size_t i = (size_t)m * nb + n + P;
    const cd num = j2[an] * a[i] + h[an] * beta[i];
    gam[i] = fabs(jp[an]) > 1e-300 ? (1.0 / jp[an]) * num : cd{0, 0};
  }
}

__global__ void incoming_kernel(int n, const cd* t, const cd* l, const cd* a0, cd* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = t[i] - l[i] + a0[i];
}

}  // namespace

extern "C" grt_status grt_eval_field(grt_ctx* c0, int64_t rhs, const void* beta_dev,
                                     int64_t n_pts, const double* xy_host, double* u_host) {
  if (!c0) return GRT_EINVAL;
  if (!c0->built) return set_err(c0, GRT_ESTATE, "grt_eval_field before grt_build");
  if (rhs < 0 || rhs >= c0->n_rhs) return set_err(c0, GRT_EINVAL, "rhs out of range");
  if (rhs > 0) {
    grt_ctx* cr = c0->rhs[(size_t)rhs - 1];
    const grt_status st = grt_eval_field(cr, 0, beta_dev, n_pts, xy_host, u_host);
    return st == GRT_OK ? st : set_err(c0, st, cr->err);
  }
  grt_ctx* c = c0;
  if (has_shapes(c))
    return set_err(c, GRT_EUNSUP, "field evaluation takes disks only (interior expansions)");
  if (c->g.te) return set_err(c, GRT_EUNSUP, "field evaluation is written for TM");
  if (c->g.curved)
    return set_err(c, GRT_EUNSUP, "field evaluation is written for flat interfaces");
  if (c->lossy)
    return set_err(c, GRT_EUNSUP, "field evaluation is written for lossless disks");
  if (c->g.k_im[2] != 0.0)
    return set_err(c, GRT_EUNSUP, "field evaluation is written for a lossless substrate");
  if (n_pts < 0 || n_pts > ((int64_t)1 << 30)) return set_err(c, GRT_EINVAL, "bad point count");
  if (n_pts == 0) return GRT_OK;
  if (!xy_host || !u_host) return set_err(c, GRT_EINVAL, "null point or output array");
  if (c->M > 0 && !beta_dev) return set_err(c, GRT_EINVAL, "null beta");
  if (c->P > 40) return set_err(c, GRT_EUNSUP, "P above 40");
  for (int64_t i = 0; i < 2 * n_pts; ++i)
    if (!std::isfinite(xy_host[i]) || std::fabs(xy_host[i]) > 1e6)
      return set_err(c, GRT_EINVAL, "non-finite point or |coordinate| > 1e6");
  hipSetDevice(c->device);
  hipStream_t s = c->stream;
  const int na = c->g.n_alpha;
  const int64_t nbeta = c->n_beta;
  cd *alpha = nullptr, *W = nullptr, *tA = nullptr, *tL = nullptr, *t0 = nullptr, *gam = nullptr,
     *dout = nullptr;
  double* dxy = nullptr;
  grt_status st = GRT_OK;
  auto fail = [&](const char* what, hipError_t e) {
    st = set_err(c, GRT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  const size_t nb_alloc = (size_t)std::max<int64_t>(1, nbeta);
  if ((e = hipMalloc(&alpha, sizeof(cd) * na)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&W, sizeof(cd) * (size_t)na * std::max(1, c->rank))) != hipSuccess)
    fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&tA, sizeof(cd) * nb_alloc)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&tL, sizeof(cd) * nb_alloc)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&t0, sizeof(cd) * nb_alloc)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&gam, sizeof(cd) * nb_alloc)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&dout, sizeof(cd) * n_pts)) != hipSuccess) fail("hipMalloc", e);
  if (st == GRT_OK && (e = hipMalloc(&dxy, sizeof(double) * 2 * n_pts)) != hipSuccess)
    fail("hipMalloc", e);
  const cd* beta = static_cast<const cd*>(beta_dev);
  if (st == GRT_OK) st = alpha_full(c, beta, alpha, W);
  if (st == GRT_OK && c->M > 0) {
    st = apply_T_only(c, beta, tA);
    if (st == GRT_OK) st = apply_lowrank_only(c, beta, tL);
    if (st == GRT_OK) st = incident_alpha(c, t0);
    if (st == GRT_OK) {
      incoming_kernel<<<(unsigned)((nbeta + 255) / 256), 256, 0, s>>>((int)nbeta, tA, tL, t0, tA);
      interior_kernel<<<(unsigned)((c->M + 63) / 64), 64, 0, s>>>(
          (int)c->M, c->P, c->g.k[1], c->d_rad, c->d_kp, tA, beta, gam);
    }
  }
  if (st == GRT_OK &&
      (e = hipMemcpyAsync(dxy, xy_host, sizeof(double) * 2 * n_pts, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    fail("hipMemcpyAsync", e);
  if (st == GRT_OK) {
    FieldIn in{};
    in.g = c->g;
    in.alpha = alpha;
    in.beta = beta;
    in.gam = gam;
    in.cx = c->d_cx;
    in.cy = c->d_cy;
    in.rad = c->d_rad;
    in.kp = c->d_kp;
    in.htab = c->d_htab;
    in.k1cos = c->g.k[0] * std::cos(c->inc.phi);
    field_kernel<<<(unsigned)((n_pts + 63) / 64), 64, 0, s>>>(in, (int)n_pts, dxy, dout);
    if ((e = hipGetLastError()) != hipSuccess) fail("field_kernel", e);
  }
  if (st == GRT_OK &&
      (e = hipMemcpyAsync(u_host, dout, sizeof(cd) * n_pts, hipMemcpyDeviceToHost, s)) != hipSuccess)
    fail("hipMemcpyAsync", e);
  if (st == GRT_OK && (e = hipStreamSynchronize(s)) != hipSuccess) fail("hipStreamSynchronize", e);
  hipStreamSynchronize(s);
  for (void* ptr : {(void*)alpha, (void*)W, (void*)tA, (void*)tL, (void*)t0, (void*)gam, (void*)dout,
                    (void*)dxy})
    if (ptr) hipFree(ptr);
  return st;
}
