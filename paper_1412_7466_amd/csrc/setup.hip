// Device-side construction of everything the apply needs (paper sec. 3, 4.1, 5).
//
//  * the rectangular empty-structure matrix A of eq. matA, one thread per entry:
//    layer potentials summed over the copies l = -1, 0, 1 with phases alpha^l
//    (eqs. repre1-repre3) on flat or curved (graph) interfaces, the
//    same-interface kernel differences (S, D, N, T of the layers on both sides) with
//    zeta-corrected trapezoid weights per target (the paper's locally corrected
//    Nystrom rule, in the graphs' parameter x), J-expansion columns, wall
//    discrepancies in the cancelled form alpha u(L) - u(L+d) =
//    alpha^2 Phi(L-d) - alpha^{-1} Phi(L+2d), Rayleigh-Bloch columns (eq. bound3);
//  * unit-norm column equilibration, SVD by rocSOLVER, truncated Sigma^+ and the
//    three factor blocks the apply streams (eq. applypA: A^+ g = V Sigma^+ U^* g);
//  * the Mie (single-disk) scattering coefficients (sec. 4.1);
//  * the L2L table J_m(k_2 rho_j) e^{i m phi_j} of every inclusion about the middle
//    J centre (Graf's theorem for J);
//  * the incident data f of eq. Arhs.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

// ---------------------------------------------------------------------------
// quadrature nodes and correction weights
// ---------------------------------------------------------------------------

// Gauss-Legendre nodes of order n on [a, b], ascending (Newton on P_n from the
// Chebyshev-like initial guess).
__global__ void gl_nodes_kernel(int n, double a, double b, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = cos(GRT_PI * (i + 0.75) / (n + 0.5));
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? x : p1, pm = (n == 1) ? 1.0 : p0;
    double dp = n * (x * pn - pm) / (x * x - 1.0);
    double dx = pn / dp;
    x -= dx;
    if (fabs(dx) < 1e-16) break;
  }
  // roots from the guess above come largest first; store ascending
  out[i] = 0.5 * (a + b) + 0.5 * (b - a) * (-x);
}

// zeta(s) for s >= 3 by direct summation with an Euler-Maclaurin tail.
__device__ double zeta_odd(double s) {
  const int Nz = 100;
  double acc = 0.0;
  for (int n = Nz - 1; n >= 1; --n) acc += pow((double)n, -s);
  double Nd = Nz;
  acc += pow(Nd, 1.0 - s) / (s - 1.0) + 0.5 * pow(Nd, -s) + s * pow(Nd, -s - 1.0) / 12.0 -
         s * (s + 1.0) * (s + 2.0) * pow(Nd, -s - 3.0) / 720.0;
  return acc;
}

// Single thread: Fornberg finite-difference weights on the stencil -K..K (unit
// spacing) combined with the zeta coefficients of the locally corrected trapezoid
// rule for K(s) = phi(s) ln|s| + psi(s):
//   zcw[p] = sum_k 2 zeta'(-2k)/(2k)! c^{(2k)}_p,  2 zeta'(-2k)/(2k)! = (-1)^k zeta(2k+1) / (2 pi)^{2k},
// so that the correction weights of a target are (the term of order 2k is
// zc_k hs^{2k+1} (phi tau)^{(2k)}(0) and the unit-spacing differences carry hs^{-2k})
//   w_p = hs zcw[p] phi(p hs) + [p = 0] hs (psi(0) + phi(0) ln(hs / 2 pi)).
__global__ void zeta_stencil_kernel(int K, double* zcw) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = 2 * K + 1;
  const int m = 2 * K;
  double z[33];
  double c[33][33];  // c[q][j]
  for (int j = 0; j < n; ++j) z[j] = (double)(j - K);
  for (int q = 0; q <= m; ++q)
    for (int j = 0; j < n; ++j) c[q][j] = 0.0;
  double c1 = 1.0, c4 = z[0];
  c[0][0] = 1.0;
  for (int i = 1; i < n; ++i) {
    int mn = i < m ? i : m;
    double c2 = 1.0, c5 = c4;
    c4 = z[i];
    for (int j = 0; j < i; ++j) {
      double c3 = z[i] - z[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k) c[k][i] = c1 * (k * c[k - 1][i - 1] - c5 * c[k][i - 1]) / c2;
        c[0][i] = -c1 * c5 * c[0][i - 1] / c2;
      }
      for (int k = mn; k >= 1; --k) c[k][j] = (c4 * c[k][j] - k * c[k - 1][j]) / c3;
      c[0][j] = c4 * c[0][j] / c3;
    }
    c1 = c2;
  }
  for (int j = 0; j < n; ++j) {
    double acc = 0.0;
    for (int k = 1; k <= K; ++k) {
      double sgn = (k & 1) ? -1.0 : 1.0;
      acc += sgn * zeta_odd(2.0 * k + 1.0) / pow(2.0 * GRT_PI, 2.0 * k) * c[2 * k][j];
    }
    zcw[j] = acc;
  }
}

// The four same-interface kernel differences per unit of the source parameter x
// (kind 0: wa S_a - wb S_b, 1: wa D_a - wb D_b, 2: N_a - N_b, 3: T_a - T_b) at
// R = target - source (r > 0), target normal ns, source normal nt, source speed spd:
//   S = (i/4)(wa H0_a - wb H0_b)
//   D = (i/4)(wa ka H1_a - wb kb H1_b)(R.n_t)/r
//   N = -(i/4)(ka H1_a - kb H1_b)(R.n_s)/r
//   T = (i/4)[(ka H1_a - kb H1_b)(n_s.n_t)/r - (ka^2 H2_a - kb^2 H2_b)(R.n_s)(R.n_t)/r^2]
// each times spd.  With logc, the coefficient phi of ln|s - t| instead: (i/4) H_n
// replaced by -J_n / (2 pi) (the log part of Y_n).
__device__ cd curve_kernel(int kind, bool logc, cd ka, cd kb, cd wa, cd wb,
                           double Rx, double Ry, double snx, double sny, double tnx, double tny,
                           double spd) {
  const double r = sqrt(Rx * Rx + Ry * Ry);
  cd Za[3], Zb[3];
  const cd ks[2] = {ka, kb};
  for (int w = 0; w < 2; ++w) {
    cd* Z = w ? Zb : Za;
    const cd z = r * ks[w];
    const cd two_z = cdiv(cd{2.0, 0.0}, z);
    if (logc) {
      cd j0, j1;
      if (z.i == 0.0) {
        double a, b, c, e;
        bessel01(z.r, a, b, c, e);
        j0 = cd{a, 0.0};
        j1 = cd{b, 0.0};
      } else {
        cd y0, y1;
        bessel01_c(z, j0, j1, y0, y1);
      }
      const double c = -1.0 / (2.0 * GRT_PI);
      Z[0] = c * j0;
      Z[1] = c * j1;
      Z[2] = c * (two_z * j1 - j0);
    } else {
      cd h0, h1;
      hankel01_c(z, h0, h1);
      Z[0] = times_i(0.25 * h0);
      Z[1] = times_i(0.25 * h1);
      Z[2] = times_i(0.25 * (two_z * h1 - h0));
    }
  }
  const double Rs = Rx * snx + Ry * sny, Rt = Rx * tnx + Ry * tny;
  cd v;
  switch (kind) {
    case 0: v = wa * Za[0] - wb * Zb[0]; break;
    case 1: v = (Rt / r) * (wa * (ka * Za[1]) - wb * (kb * Zb[1])); break;
    case 2: v = (-Rs / r) * (ka * Za[1] - kb * Zb[1]); break;
    default:
      v = ((snx * tnx + sny * tny) / r) * (ka * Za[1] - kb * Zb[1]) -
          (Rs * Rt / (r * r)) * ((ka * ka) * Za[2] - (kb * kb) * Zb[2]);
  }
  return spd * v;
}

// (phi(0), psi(0)) of the four kernel differences at a node of speed spd with
// curvature term f2 = f'' (ln r = ln|s - t| + ln spd + O(s - t); the k-free singular
// parts cancel in the differences except for the weighted double layer, whose
// (R.n_t)/(2 pi r^2) tends to f'' / (4 pi spd^3)):
//   S: phi0 = -(wa - wb) spd / (2 pi),
//      psi0 = spd [(wa - wb)(i/4 - gamma/(2 pi) - ln(spd)/(2 pi)) - (wa ln(ka/2) - wb ln(kb/2))/(2 pi)]
//   D: phi0 = 0, psi0 = (wa - wb) f'' / (4 pi spd^2);  N: phi0 = psi0 = 0
//   T: phi0 = -(ka^2 - kb^2) spd / (4 pi),
//      psi0 = spd [i (ka^2 - kb^2)/8 - (ka^2 ln(ka/2) - kb^2 ln(kb/2))/(4 pi)
//                  + (ka^2 - kb^2)(1 - 2 gamma)/(8 pi) - (ka^2 - kb^2) ln(spd)/(4 pi)]
// (small-argument series of J_n, Y_n).
__device__ void curve_limits(int kind, cd ka, cd kb, cd wa, cd wb, double spd,
                             double f2, cd& phi0, cd& psi0) {
  const double gam = GRT_EULER_GAMMA, pi = GRT_PI, lsp = log(spd);
  const cd d2 = ka * ka - kb * kb;
  // principal ln(k / 2) (complex for an absorbing layer)
  const cd la{log(0.5 * sqrt(cabs2(ka))), atan2(ka.i, ka.r)};
  const cd lb{log(0.5 * sqrt(cabs2(kb))), atan2(kb.i, kb.r)};
  switch (kind) {
    case 0:
      phi0 = (-spd / (2.0 * pi)) * (wa - wb);
      psi0 = spd * (cd{-gam / (2.0 * pi) - lsp / (2.0 * pi), 0.25} * (wa - wb) -
                    (1.0 / (2.0 * pi)) * (wa * la - wb * lb));
      break;
    case 1:
      phi0 = cd{0.0, 0.0};
      psi0 = (f2 / (4.0 * pi * spd * spd)) * (wa - wb);
      break;
    case 2:
      phi0 = cd{0.0, 0.0};
      psi0 = cd{0.0, 0.0};
      break;
    default:
      phi0 = (-spd / (4.0 * pi)) * d2;
      psi0 = spd * ((-1.0 / (4.0 * pi)) * ((ka * ka) * la - (kb * kb) * lb) +
                    ((1.0 - 2.0 * gam) / (8.0 * pi) - lsp / (4.0 * pi)) * d2 +
                    times_i(0.125 * d2));
  }
}

// Wavenumbers and layer weights of interface `line`'s same-interface blocks: the
// layers above and below it; the single and double layers carry pv of their layer
// (TE: eps), the flux rows' N and T parts are unweighted (fl pv = 1).
__device__ __forceinline__ cd layer_k(const DevGeom& g, int l) { return cd{g.k[l], g.k_im[l]}; }

// TE layer factors as complex numbers (complex for the absorbing substrate's eps_3)
__device__ __forceinline__ cd layer_pv(const DevGeom& g, int l) { return cd{g.pv[l], g.pv_im[l]}; }
__device__ __forceinline__ cd layer_fl(const DevGeom& g, int l) { return cd{g.fl[l], g.fl_im[l]}; }

__device__ __forceinline__ void line_pair(const DevGeom& g, int line, int kind, cd& ka,
                                          cd& kb, cd& wa, cd& wb) {
  ka = layer_k(g, line);
  kb = layer_k(g, line + 1);
  const bool weighted = kind < 2;
  wa = weighted ? layer_pv(g, line) : cd{1.0, 0.0};
  wb = weighted ? layer_pv(g, line + 1) : cd{1.0, 0.0};
}

// Correction weights of every target: one thread per (interface, target), all four
// kinds; phi at the stencil nodes i + p (wrapping onto the copies l = -1, +1), then
//   w_p = hs zcw[p] phi_p + [p = 0] hs (psi(0) + phi(0) ln(hs / 2 pi)).
// The Bloch phase of a wrapped node is applied where the weight is used.
__global__ void curve_weights_kernel(DevGeom g, const double* zcw, cd* w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N, K = g.zeta_K, n = 2 * K + 1;
  if (t >= 2 * N) return;
  const int line = t / N, i = t - line * N;
  const double* ni = g.node + ((size_t)line * N + i) * NODE_STRIDE;
  const double lhs = log(g.hs / (2.0 * GRT_PI));
  for (int kind = 0; kind < 4; ++kind) {
    cd ka, kb, wa, wb, phi0, psi0;
    line_pair(g, line, kind, ka, kb, wa, wb);
    curve_limits(kind, ka, kb, wa, wb, ni[4], ni[5], phi0, psi0);
    cd* out = w + (((size_t)line * 4 + kind) * N + i) * n;
    for (int p = -K; p <= K; ++p) {
      cd ph;
      if (p == 0) {
        ph = phi0;
      } else {
        const int gi = i + p;
        const int l = gi < 0 ? -1 : (gi >= N ? 1 : 0);
        const double* nj = g.node + ((size_t)line * N + gi - l * N) * NODE_STRIDE;
        ph = curve_kernel(kind, true, ka, kb, wa, wb, ni[0] - (nj[0] + l * g.d), ni[1] - nj[1],
                          ni[2], ni[3], nj[2], nj[3], nj[4]);
      }
      cd wp = (g.hs * zcw[p + K]) * ph;
      if (p == 0) wp += g.hs * (psi0 + lhs * phi0);
      out[p + K] = wp;
    }
  }
}

// ---------------------------------------------------------------------------
// matrix entries
// ---------------------------------------------------------------------------

__device__ __forceinline__ cd alpha_pow(const DevGeom& g, int l) {
  if (l == 0) return cd{1.0, 0.0};
  cd r = (l > 0) ? g.alpha : g.alpha_inv;
  int a = l > 0 ? l : -l;
  cd o{1.0, 0.0};
  for (int t = 0; t < a; ++t) o = o * r;
  return o;
}

// Single-layer G = (i/4) H0(kr) and double-layer dG/dn_y = (ik/4) H1(kr) (R.n)/r
// (source normal n = (nx, ny)), R = target - source; with deriv, their derivatives
// along the unit direction (tx, ty) at the target:
//   dS = -(ik/4) H1 (R.t)/r,  dD = (ik/4) [-k H2 (R.n)(R.t)/r^2 + H1 (n.t) / r].
__device__ void lp_kernels(cd k, double Rx, double Ry, double nx, double ny, bool deriv,
                           double tx, double ty, cd& S, cd& D) {
  double r = sqrt(Rx * Rx + Ry * Ry);
  const cd z = r * k;
  cd h0, h1;
  hankel01_c(z, h0, h1);
  const double Rn = Rx * nx + Ry * ny;
  const cd kh1 = k * h1;
  if (!deriv) {
    S = times_i(0.25 * h0);
    D = times_i((0.25 * Rn / r) * kh1);
    return;
  }
  cd h2 = cdiv(cd{2.0, 0.0}, z) * h1 - h0;
  double Rt = Rx * tx + Ry * ty;
  S = times_i((-0.25 * Rt / r) * kh1);
  D = times_i(0.25 * ((-Rn * Rt / (r * r)) * (k * (k * h2)) + ((nx * tx + ny * ty) / r) * kh1));
}

__device__ __forceinline__ const double* node_at(const DevGeom& g, int line, int j) {
  return g.node + ((size_t)line * g.N + j) * NODE_STRIDE;
}

// Three-copy trapezoid sum from node j of interface `line` (arc-length weight
// hs * speed).
__device__ void three_copy(const DevGeom& g, cd k, double tx, double ty, int line, int j,
                           bool deriv, double dx, double dy, cd& S, cd& D) {
  const double* nj = node_at(g, line, j);
  S = cd{0, 0};
  D = cd{0, 0};
  for (int l = -1; l <= 1; ++l) {
    cd a, b;
    lp_kernels(k, tx - (nj[0] + l * g.d), ty - nj[1], nj[2], nj[3], deriv, dx, dy, a, b);
    cd w = alpha_pow(g, l);
    S += w * a;
    D += w * b;
  }
  const double wq = g.hs * nj[4];
  S = wq * S;
  D = wq * D;
}

// Wall discrepancy alpha u(L) - u(R) of the three copies of node j, cancelled:
// alpha^2 Phi(-3d/2, y) - alpha^{-1} Phi(3d/2, y), Phi the l = 0 copy.
__device__ void wall_cancelled(const DevGeom& g, cd k, double y, int line, int j, bool deriv,
                               cd& S, cd& D) {
  const double* nj = node_at(g, line, j);
  cd a1, b1, a2, b2;
  lp_kernels(k, -1.5 * g.d - nj[0], y - nj[1], nj[2], nj[3], deriv, 1.0, 0.0, a1, b1);
  lp_kernels(k, 1.5 * g.d - nj[0], y - nj[1], nj[2], nj[3], deriv, 1.0, 0.0, a2, b2);
  cd w1 = g.alpha * g.alpha, w2 = -g.alpha_inv;
  const double wq = g.hs * nj[4];
  S = wq * (w1 * a1 + w2 * a2);
  D = wq * (w1 * b1 + w2 * b2);
}

// Same-interface block entry (target node i, source node j) of interface `line`,
// kind 0..3 (weighted S, weighted D, N, T differences): punctured three-copy
// trapezoid sum plus the target's stencil corrections.
__device__ cd self_entry(const DevGeom& g, int line, int kind, int i, int j) {
  cd ka, kb, wa, wb;
  line_pair(g, line, kind, ka, kb, wa, wb);
  const int N = g.N, K = g.zeta_K;
  const double* ni = node_at(g, line, i);
  const double* nj = node_at(g, line, j);
  const cd* wc = g.wcorr + (((size_t)line * 4 + kind) * N + i) * (2 * K + 1);
  cd acc{0, 0};
  for (int l = -1; l <= 1; ++l) {
    cd w = alpha_pow(g, l);
    if (!(l == 0 && i == j)) {
      cd kv = curve_kernel(kind, false, ka, kb, wa, wb, ni[0] - (nj[0] + l * g.d), ni[1] - nj[1],
                           ni[2], ni[3], nj[2], nj[3], nj[4]);
      acc += g.hs * (w * kv);
    }
    int p = j + l * N - i;
    if (p >= -K && p <= K) acc += w * wc[p + K];
  }
  return acc;
}

// J-expansion column q of layer `lay` at target (tx, ty): J_q(k r) e^{i q theta}
// or its derivative along (dx, dy) from (d_x +- i d_y) Z_q e^{iq theta} =
// -+ k Z_{q+-1} e^{i(q+-1) theta}.
__device__ cd jcol(const DevGeom& g, int lay, int q, double tx, double ty, bool deriv, double dx,
                   double dy) {
  const cd k = layer_k(g, lay);
  double vx = tx, vy = ty - g.jcy[lay];
  double r = sqrt(vx * vx + vy * vy);
  cd jm, j0, jp;
  if (k.i == 0.0) {
    double a, b, c;
    bessel_j_three(k.r * r, q, a, b, c);
    jm = cd{a, 0.0};
    j0 = cd{b, 0.0};
    jp = cd{c, 0.0};
  } else {
    bessel_j_three_c(r * k, q, jm, j0, jp);
  }
  cd e = (r > 0) ? cd{vx / r, vy / r} : cd{1.0, 0.0};
  auto epow = [&](int n) { return n >= 0 ? cpowi(e, n) : cpowi(conj(e), -n); };
  if (!deriv) return j0 * epow(q);
  cd fm = jm * epow(q - 1), fp = jp * epow(q + 1);
  cd gx = 0.5 * (k * (fm - fp));
  cd gy = times_i(0.5 * (k * (fm + fp)));
  return dx * gx + dy * gy;
}

// sqrt(k^2 - kap^2): non-negative real or positive imaginary part for real k; for an
// absorbing layer (Im k > 0, so Im(k^2 - kap^2) > 0) the principal root, with positive
// real and imaginary parts (the Rayleigh-Bloch wave decays away from the layers).
__device__ cd kz_branch(cd k, double kap) {
  if (k.i == 0.0) {
    double v = k.r * k.r - kap * kap;
    return v >= 0 ? cd{sqrt(v), 0.0} : cd{0.0, sqrt(-v)};
  }
  return csqrt_principal(k * k - cd{kap * kap, 0.0});
}

__device__ cd A_entry(const DevGeom& g, int row, int col) {
  int rb = 0;
  while (row >= g.row_off[rb + 1]) ++rb;
  int cb = 0;
  while (col >= g.col_off[cb + 1]) ++cb;
  int i = row - g.row_off[rb];
  int j = col - g.col_off[cb];
  const double d = g.d;
  const cd k1 = layer_k(g, 0), k2 = layer_k(g, 1), k3 = layer_k(g, 2);
  cd S, D;
  cd zero{0, 0};
  switch (rb) {
    case RB_G1V:
    case RB_G1N: {
      bool dv = (rb == RB_G1N);
      const double* ni = node_at(g, 0, i);
      const double tx = ni[0], ty = ni[1], nx = ni[2], ny = ni[3];
      // layer factors: potentials of layer l carry pv[l]; flux rows take fl[l] of the
      // field of layer l (the self blocks' N, T and identity parts are unchanged)
      switch (cb) {
        case CB_MU1:
          return dv ? self_entry(g, 0, 3, i, j)
                    : (i == j ? cd{0.5 * (g.pv[0] + g.pv[1]), 0} : zero) + self_entry(g, 0, 1, i, j);
        case CB_SIG1:
          return dv ? (i == j ? cd{-1, 0} : zero) + self_entry(g, 0, 2, i, j)
                    : self_entry(g, 0, 0, i, j);
        case CB_MU2:
        case CB_SIG2:
          three_copy(g, k2, tx, ty, 1, j, dv, nx, ny, S, D);
          return -((dv ? g.fl[1] : 1.0) * g.pv[1]) * (cb == CB_MU2 ? D : S);
        case CB_A2: return -(dv ? g.fl[1] : 1.0) * jcol(g, 1, j - g.Q[1], tx, ty, dv, nx, ny);
        case CB_A1: return (dv ? g.fl[0] : 1.0) * jcol(g, 0, j - g.Q[0], tx, ty, dv, nx, ny);
        default: return zero;
      }
    }
    case RB_G2V:
    case RB_G2N: {
      bool dv = (rb == RB_G2N);
      const double* ni = node_at(g, 1, i);
      const double tx = ni[0], ty = ni[1], nx = ni[2], ny = ni[3];
      switch (cb) {
        case CB_MU1:
        case CB_SIG1:
          three_copy(g, k2, tx, ty, 0, j, dv, nx, ny, S, D);
          return ((dv ? g.fl[1] : 1.0) * g.pv[1]) * (cb == CB_MU1 ? D : S);
        case CB_MU2:
          return dv ? self_entry(g, 1, 3, i, j)
                    : (i == j ? 0.5 * (layer_pv(g, 1) + layer_pv(g, 2)) : zero) +
                          self_entry(g, 1, 1, i, j);
        case CB_SIG2:
          return dv ? (i == j ? cd{-1, 0} : zero) + self_entry(g, 1, 2, i, j)
                    : self_entry(g, 1, 0, i, j);
        case CB_A2: return (dv ? g.fl[1] : 1.0) * jcol(g, 1, j - g.Q[1], tx, ty, dv, nx, ny);
        case CB_A3: return -((dv ? layer_fl(g, 2) : cd{1.0, 0.0}) * jcol(g, 2, j - g.Q[2], tx, ty, dv, nx, ny));
        default: return zero;
      }
    }
    case RB_W2V: case RB_W2D: case RB_W1V: case RB_W1D: case RB_W3V: case RB_W3D: {
      int lay = (rb <= RB_W2D) ? 1 : (rb <= RB_W1D ? 0 : 2);
      bool dv = (rb == RB_W2D || rb == RB_W1D || rb == RB_W3D);
      double y = g.yw[lay][i];
      const cd k = layer_k(g, lay);
      int jcb = (lay == 1) ? CB_A2 : (lay == 0 ? CB_A1 : CB_A3);
      bool top_line = (cb == CB_MU1 || cb == CB_SIG1);
      bool bot_line = (cb == CB_MU2 || cb == CB_SIG2);
      if ((top_line && lay != 2) || (bot_line && lay != 0)) {
        wall_cancelled(g, k, y, top_line ? 0 : 1, j, dv, S, D);
        return layer_pv(g, lay) * ((cb == CB_MU1 || cb == CB_MU2) ? D : S);
      }
      if (cb == jcb) {
        int q = j - g.Q[lay];
        cd L = jcol(g, lay, q, -0.5 * d, y, dv, 1.0, 0.0);
        cd R = jcol(g, lay, q, 0.5 * d, y, dv, 1.0, 0.0);
        return g.alpha * L - R;
      }
      return zero;
    }
    case RB_UV: case RB_UN: case RB_DV: case RB_DN: {
      bool upper = (rb == RB_UV || rb == RB_UN);
      bool dv = (rb == RB_UN || rb == RB_DN);
      double tx = -0.5 * d + (i + 0.5) * d / g.Nu;
      double ty = upper ? g.y0 : -g.y0;
      const cd k = upper ? k1 : k3;
      if (upper && (cb == CB_MU1 || cb == CB_SIG1)) {
        three_copy(g, k, tx, ty, 0, j, dv, 0.0, 1.0, S, D);
        return g.pv[0] * (cb == CB_MU1 ? D : S);
      }
      if (!upper && (cb == CB_MU2 || cb == CB_SIG2)) {
        three_copy(g, k, tx, ty, 1, j, dv, 0.0, 1.0, S, D);
        return layer_pv(g, 2) * (cb == CB_MU2 ? D : S);
      }
      if (upper && cb == CB_A1) return jcol(g, 0, j - g.Q[0], tx, ty, dv, 0.0, 1.0);
      if (!upper && cb == CB_A3) return jcol(g, 2, j - g.Q[2], tx, ty, dv, 0.0, 1.0);
      if ((upper && cb == CB_C) || (!upper && cb == CB_D)) {
        double kapn = g.kappa + 2.0 * GRT_PI * (g.n_rb_lo + j) / d;
        cd e = cexpi(kapn * tx);
        if (!dv) return -e;
        cd kz = kz_branch(k, kapn);
        cd ik = times_i(kz);
        return upper ? -(ik * e) : (ik * e);
      }
      return zero;
    }
    default:
      return zero;
  }
}

__global__ void assemble_A_kernel(DevGeom g, cd* A) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  int col = blockIdx.y;
  if (row >= g.n_rows || col >= g.n_alpha) return;
  A[(size_t)col * g.n_rows + row] = A_entry(g, row, col);
}

// One block per column: 2-norm, then scale the column to unit norm.
__global__ void equilibrate_kernel(cd* A, int n_rows, int n_cols, double* scale) {
  int col = blockIdx.x;
  if (col >= n_cols) return;
  cd* a = A + (size_t)col * n_rows;
  __shared__ double red[256];
  double s = 0.0;
  for (int r = threadIdx.x; r < n_rows; r += blockDim.x) s += cabs2(a[r]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double nrm = sqrt(red[0]);
  double sc = nrm > 0 ? 1.0 / nrm : 1.0;
  for (int r = threadIdx.x; r < n_rows; r += blockDim.x) a[r] = sc * a[r];
  if (threadIdx.x == 0) scale[col] = sc;
}

// W1[k][i] = conj(U[i][k]) / sigma_k (k < rank, i < n_g)
__global__ void build_W1_kernel(const cd* U, int ldu, const double* sv, int rank, int n_g, cd* W1) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= n_g || k >= rank) return;
  cd u = U[(size_t)k * ldu + i];
  W1[(size_t)k * n_g + i] = (1.0 / sv[k]) * conj(u);
}

// W[i][k] = E[i0 + i] * conj(VH[k][i0 + i]) (V = (V^H)^H, E the column scales)
__global__ void build_Wv_kernel(const cd* VH, int ldv, const double* E, int i0, int rows, int rank,
                                cd* W) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (k >= rank || i >= rows) return;
  cd v = VH[(size_t)(i0 + i) * ldv + k];
  W[(size_t)i * rank + k] = E[i0 + i] * conj(v);
}

// Mie coefficients of every disk (sec. 4.1), s_{-n} = s_n:
//   s_n = -[k2 J_n'(x) J_n(y) - kp J_n(x) J_n'(y)] / [k2 H_n'(x) J_n(y) - kp H_n(x) J_n'(y)],
// x = k2 R, y = kp R; Z_n' = Z_{n-1} - (n/x) Z_n, Z_0' = -Z_1.
// Absorbing disk (complex k_p): the same formula with J_n(y), J_n'(y) and the interior
// weight at complex y = k_p R.
__device__ void mie_disk_complex(int P, double k2, double R, cd kpc, cd* s, int te, double eps2,
                                 double omega) {
  const double x = k2 * R;
  const cd y = R * kpc;
  double jx[48];
  cd jy[48];
  bessel_jn_array(x, P + 1, jx);
  bessel_jn_array_c(y, P + 1, jy);
  cd H[48];
  hankel01(x, H[0], H[1]);
  for (int n = 1; n <= P; ++n) H[n + 1] = (2.0 * n / x) * H[n] - H[n - 1];
  const cd iy = cdiv(cd{1.0, 0.0}, y);
  const double w2 = te ? k2 / eps2 : k2;
  const cd wp = te ? cdiv(cd{omega * omega, 0.0}, kpc) : kpc;  // k_p / eps_p = omega^2 / k_p
  for (int n = 0; n <= P; ++n) {
    double djx = (n == 0) ? -jx[1] : jx[n - 1] - (n / x) * jx[n];
    cd djy = (n == 0) ? -jy[1] : jy[n - 1] - (double)n * (iy * jy[n]);
    cd dH = (n == 0) ? -H[1] : H[n - 1] - (n / x) * H[n];
    cd num = (w2 * djx) * jy[n] - jx[n] * (wp * djy);
    cd den = (w2 * jy[n]) * dH - (wp * djy) * H[n];
    cd sn = -cdiv(num, den);
    s[P + n] = sn;
    s[P - n] = sn;
  }
}

__global__ void mie_kernel(int M, int P, double k2, const double* rad, const double* kp,
                           const double* kp_im, cd* s, int te, double eps2, double omega) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  if (kp_im && kp_im[m] != 0.0) {
    mie_disk_complex(P, k2, rad[m], cd{kp[m], kp_im[m]}, s + (size_t)m * (2 * P + 1), te, eps2,
                     omega);
    return;
  }
  double R = rad[m];
  double x = k2 * R, y = kp[m] * R;
  double jx[48], jy[48];
  bessel_jn_array(x, P + 1, jx);
  bessel_jn_array(y, P + 1, jy);
  cd hprev, hcur;
  hankel01(x, hprev, hcur);  // H_0, H_1
  int nb = 2 * P + 1;
  cd H[48];
  H[0] = hprev;
  H[1] = hcur;
  for (int n = 1; n <= P; ++n) H[n + 1] = (2.0 * n / x) * H[n] - H[n - 1];
  for (int n = 0; n <= P; ++n) {
    double djx = (n == 0) ? -jx[1] : jx[n - 1] - (n / x) * jx[n];
    double djy = (n == 0) ? -jy[1] : jy[n - 1] - (n / y) * jy[n];
    cd dH = (n == 0) ? -H[1] : H[n - 1] - (n / x) * H[n];
    // TE weights the radial derivatives by 1/eps of each side
    const double w2 = te ? k2 / eps2 : k2;
    const double wp = te ? omega * omega / kp[m] : kp[m];   // kp / eps_p = omega^2 / kp
    double num = w2 * djx * jy[n] - wp * jx[n] * djy;
    cd den = (w2 * jy[n]) * dH - (wp * djy) * H[n];
    cd sn = cdiv(cd{-num, 0.0}, den);
    s[(size_t)m * nb + P + n] = sn;
    s[(size_t)m * nb + P - n] = sn;
  }
}

// Scaling of the normalised system: d[m][n] = |H_|n|(k2 R_m)|, the size of each
// outgoing multipole on its own disk boundary (upward recurrence), and 1/d.
__global__ void dnorm_kernel(int M, int P, double k2, const double* rad, double* dn,
                             double* dinv) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double x = k2 * rad[m];
  cd hp, hc;
  hankel01(x, hp, hc);
  int nb = 2 * P + 1;
  for (int q = 0; q <= P; ++q) {
    double a = sqrt(cabs2(hp));
    dn[(size_t)m * nb + P + q] = a;
    dn[(size_t)m * nb + P - q] = a;
    dinv[(size_t)m * nb + P + q] = 1.0 / a;
    dinv[(size_t)m * nb + P - q] = 1.0 / a;
    cd hn = (2.0 * (q + 1) / x) * hc - hp;
    hp = hc;
    hc = hn;
  }
}

// L2L generator of every inclusion: E_j[m] = J_m(k2 rho) e^{i m phi}, m = -L..L,
// rho e^{i phi} = c_j - (0, 0).
__global__ void l2l_table_kernel(int M, int L, double k2, const double* cx, const double* cy,
                                 cd* E) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double vx = cx[j], vy = cy[j];
  double r = sqrt(vx * vx + vy * vy);
  double jn[512];
  bessel_jn_array(k2 * r, L, jn);
  cd e = (r > 0) ? cd{vx / r, vy / r} : cd{1.0, 0.0};
  cd ep{1.0, 0.0};
  cd* row = E + (size_t)j * (2 * L + 1);
  for (int m = 0; m <= L; ++m) {
    row[L + m] = jn[m] * ep;
    double sg = (m & 1) ? -1.0 : 1.0;
    row[L - m] = (sg * jn[m]) * conj(ep);
    ep = ep * e;
  }
}

// f of eq. Arhs restricted to the Gamma_1 rows: -u_inc and -du_inc/dn at the nodes of
// Gamma_1, du_inc/dn = i (kappa n_x - k1 cos(phi) n_y) u_inc.
__global__ void rhs_f_kernel(DevGeom g, double k1cos, int n_g, cd* f) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_g) return;
  cd v{0, 0};
  if (r < 2 * g.N) {
    const double* ni = g.node + (size_t)(r % g.N) * NODE_STRIDE;
    cd ui = cexpi(g.kappa * ni[0] - k1cos * ni[1]);
    // flux row: fl0 du_inc/dn; stored divided by fl1, the factor the W1 columns of the
    // flux rows carry (so that W1 (f - C x) keeps C x in its TM form)
    v = (r < g.N) ? -ui
                  : (-g.fl[0] / g.fl[1]) * times_i((g.kappa * ni[2] - k1cos * ni[3]) * ui);
  }
  f[r] = v;
}

// TE: the flux rows of C x take 1/eps_2 (folded into the columns of W1 for those
// rows) and the middle layer's potentials carry eps_2 (folded into the rows of W2 for
// the interface densities), so the apply kernels keep their TM form.
__global__ void te_fold_kernel(cd* W1, int rank, int n_g, cd* W2, int n_b, int n_dens, int N,
                               double fl1, double pv1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (k >= rank) return;
  if (i < n_g && ((i >= N && i < 2 * N) || (i >= 3 * N && i < 4 * N)))
    W1[(size_t)k * n_g + i] = fl1 * W1[(size_t)k * n_g + i];
  if (i < n_b && i < n_dens) W2[(size_t)i * rank + k] = pv1 * W2[(size_t)i * rank + k];
}

// y[i] = sum_k W[i][k] x[k], one 64-lane wavefront per row.
__global__ void __launch_bounds__(256) gemv_rows_kernel(const cd* __restrict__ W,
                                                        const cd* __restrict__ x, cd* y, int rows,
                                                        int cols) {
  int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (wave >= rows) return;
  const cd* w = W + (size_t)wave * cols;
  // four independent partial sums: four row segments in flight per lane
  double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
  int k = lane;
  for (; k + 192 < cols; k += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const cd a = w[k + 64 * u], b = x[k + 64 * u];
      ar[u] = fma(a.r, b.r, ar[u]);
      ar[u] = fma(-a.i, b.i, ar[u]);
      ai[u] = fma(a.r, b.i, ai[u]);
      ai[u] = fma(a.i, b.r, ai[u]);
    }
  }
  for (; k < cols; k += 64) {
    const cd a = w[k], b = x[k];
    ar[0] = fma(a.r, b.r, ar[0]);
    ar[0] = fma(-a.i, b.i, ar[0]);
    ai[0] = fma(a.r, b.i, ai[0]);
    ai[0] = fma(a.i, b.r, ai[0]);
  }
  double sr = (ar[0] + ar[1]) + (ar[2] + ar[3]), si = (ai[0] + ai[1]) + (ai[2] + ai[3]);
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (lane == 0) y[wave] = cd{sr, si};
}

// One thread per interval of the H_0, H_1 interpolation table.
__global__ void htab_kernel(double* tab) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < HTAB_NI) htab_interval(k, tab + k * HTAB_STRIDE);
}

}  // namespace

void launch_build_Wv(hipStream_t s, const grt_ctx* c, int i0, int rows, cd* W) {
  dim3 g((c->rank + 255) / 256, rows);
  build_Wv_kernel<<<g, 256, 0, s>>>(c->d_VH, c->g.n_alpha, c->d_colscale, i0, rows, c->rank, W);
}

void launch_gemv_rows(hipStream_t s, const cd* W, const cd* x, cd* y, int rows, int cols) {
  if (rows <= 0) return;
  int blocks = (rows + 3) / 4;
  gemv_rows_kernel<<<blocks, 256, 0, s>>>(W, x, y, rows, cols);
}

static grt_status rocblas_err(grt_ctx* c, const char* what, int st) {
  return set_err(c, GRT_EHIP, std::string(what) + " failed with rocBLAS status " + std::to_string(st));
}

// ---------------------------------------------------------------------------
// Sharing of the layer factors.  A, its SVD and the factor blocks depend only on
// the layered structure, its discretization, omega and phi (not on the
// inclusions), so problems that agree on those share one set, found through a
// process-wide cache of weak references (freed with the last context using it).
// ---------------------------------------------------------------------------
LayerFactors::~LayerFactors() {
  hipSetDevice(device);
  void* p[] = {yw, node, colscale, sv, htab, wcorr, A, U, VH, W1, W2, W3, f};
  for (void* q : p)
    if (q) hipFree(q);
}

static std::string layer_key(const grt_ctx* c) {
  const grt_layers& L = c->lay;
  std::vector<double> v = {L.d, L.h, L.y0, L.n_layer[0], L.n_layer[1], L.n_layer[2], L.pinv_eps,
                           c->inc.omega, c->inc.phi, L.n3_im};
  std::vector<int> iv = {c->device, L.N, L.Nw[0], L.Nw[1], L.Nw[2], L.Q[0], L.Q[1], L.Q[2], L.Nu,
                         L.n_rb_lo, L.Nrb, L.zeta_K, c->g.te};
  std::string k(reinterpret_cast<const char*>(v.data()), v.size() * sizeof(double));
  k.append(reinterpret_cast<const char*>(iv.data()), iv.size() * sizeof(int));
  const int F = (int)(c->hiface.size() / 4);
  k.append(reinterpret_cast<const char*>(&F), sizeof(int));
  k.append(reinterpret_cast<const char*>(c->hiface.data()), c->hiface.size() * sizeof(double));
  return k;
}

static std::mutex g_cache_mu;
static std::map<std::string, std::weak_ptr<LayerFactors>> g_cache;

static void attach_factors(grt_ctx* c, const std::shared_ptr<LayerFactors>& lf) {
  c->lf = lf;
  c->d_yw = lf->yw;
  c->d_node = lf->node;
  c->g.node = lf->node;
  c->d_colscale = lf->colscale;
  c->d_sv = lf->sv;
  c->d_htab = lf->htab;
  c->d_wcorr = lf->wcorr;
  c->d_A = lf->A;
  c->d_U = lf->U;
  c->d_VH = lf->VH;
  c->d_W1 = lf->W1;
  c->d_W2 = lf->W2;
  c->d_W3 = lf->W3;
  c->d_f = lf->f;
  c->rank = lf->rank;
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    c->g.yw[l] = lf->yw + off;
    off += c->g.Nw[l];
  }
  c->g.wcorr = lf->wcorr;
}

static grt_status build_layers(grt_ctx* c);
static grt_status build_inclusions(grt_ctx* c);

grt_status setup_build(grt_ctx* c) {
  const std::string key = layer_key(c);
  std::shared_ptr<LayerFactors> lf;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) lf = it->second.lock();
  }
  if (lf) {
    attach_factors(c, lf);
  } else {
    grt_status st = build_layers(c);
    if (st != GRT_OK) return st;
    lf = std::make_shared<LayerFactors>();
    lf->device = c->device;
    lf->yw = c->d_yw;
    lf->node = c->d_node;
    lf->colscale = c->d_colscale;
    lf->sv = c->d_sv;
    lf->htab = c->d_htab;
    lf->wcorr = c->d_wcorr;
    lf->A = c->d_A;
    lf->U = c->d_U;
    lf->VH = c->d_VH;
    lf->W1 = c->d_W1;
    lf->W2 = c->d_W2;
    lf->W3 = c->d_W3;
    lf->f = c->d_f;
    lf->rank = c->rank;
    c->lf = lf;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();)
      it = it->second.expired() ? g_cache.erase(it) : std::next(it);
    g_cache[key] = lf;
  }
  return build_inclusions(c);
}

// Only what the translation needs: the H_0 / H_1 table (the context's own) and the
// inclusion data (Mie diagonal, normalisation).  No layered structure.
grt_status setup_translation(grt_ctx* c) {
  GRT_HIP(c, hipMalloc(&c->d_htab, sizeof(double) * HTAB_SIZE));
  htab_kernel<<<1, 64, 0, c->stream>>>(c->d_htab);
  GRT_HIP(c, hipGetLastError());
  return build_inclusions(c);
}

static grt_status build_layers(grt_ctx* c) {
  hipStream_t s = c->stream;
  DevGeom& g = c->g;
  const int K = g.zeta_K;
  // wall nodes
  const int nwt = g.Nw[0] + g.Nw[1] + g.Nw[2];
  GRT_HIP(c, hipMalloc(&c->d_yw, sizeof(double) * nwt));
  // interface nodes: x cell-centred, the graphs' heights, normals, speeds and f''
  // (host arithmetic on the Fourier coefficients, O(N F))
  const int F = (int)(c->hiface.size() / 4);
  {
    std::vector<double> nd((size_t)2 * g.N * NODE_STRIDE);
    for (int line = 0; line < 2; ++line)
      for (int i = 0; i < g.N; ++i) {
        const double x = -0.5 * g.d + (i + 0.5) * g.hs;
        const double* co = c->hiface.data();
        const double f0 = F ? iface_height(co, F, line, g.h, g.d, x, 0) : (line ? -g.h : g.h);
        const double f1 = F ? iface_height(co, F, line, g.h, g.d, x, 1) : 0.0;
        const double f2 = F ? iface_height(co, F, line, g.h, g.d, x, 2) : 0.0;
        const double sp = std::sqrt(1.0 + f1 * f1);
        double* o = nd.data() + ((size_t)line * g.N + i) * NODE_STRIDE;
        o[0] = x;
        o[1] = f0;
        o[2] = -f1 / sp;
        o[3] = 1.0 / sp;
        o[4] = sp;
        o[5] = f2;
      }
    GRT_HIP(c, hipMalloc(&c->d_node, sizeof(double) * nd.size()));
    GRT_HIP(c, hipMemcpyAsync(c->d_node, nd.data(), sizeof(double) * nd.size(),
                              hipMemcpyHostToDevice, s));
    GRT_HIP(c, hipStreamSynchronize(s));  // nd is a host temporary
    g.node = c->d_node;
  }
  // the walls end on the interfaces at x = +-d/2
  const double e1 = F ? iface_height(c->hiface.data(), F, 0, g.h, g.d, 0.5 * g.d, 0) : g.h;
  const double e2 = F ? iface_height(c->hiface.data(), F, 1, g.h, g.d, 0.5 * g.d, 0) : -g.h;
  double spans[3][2] = {{e1, g.y0}, {e2, e1}, {-g.y0, e2}};
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    gl_nodes_kernel<<<(g.Nw[l] + 63) / 64, 64, 0, s>>>(g.Nw[l], spans[l][0], spans[l][1],
                                                        c->d_yw + off);
    g.yw[l] = c->d_yw + off;
    off += g.Nw[l];
  }
  GRT_HIP(c, hipMalloc(&c->d_htab, sizeof(double) * HTAB_SIZE));
  htab_kernel<<<1, 64, 0, s>>>(c->d_htab);
  // per-target correction weights of the same-interface blocks
  {
    double* zcw = nullptr;
    GRT_HIP(c, hipMalloc(&zcw, sizeof(double) * (2 * K + 1)));
    zeta_stencil_kernel<<<1, 64, 0, s>>>(K, zcw);
    GRT_HIP(c, hipMalloc(&c->d_wcorr, sizeof(cd) * (size_t)8 * g.N * (2 * K + 1)));
    curve_weights_kernel<<<(2 * g.N + 127) / 128, 128, 0, s>>>(g, zcw, c->d_wcorr);
    GRT_HIP(c, hipGetLastError());
    GRT_HIP(c, hipStreamSynchronize(s));
    hipFree(zcw);
  }
  g.wcorr = c->d_wcorr;

  // A, equilibrated
  const size_t nA = (size_t)g.n_rows * g.n_alpha;
  GRT_HIP(c, hipMalloc(&c->d_A, sizeof(cd) * nA));
  GRT_HIP(c, hipMalloc(&c->d_colscale, sizeof(double) * g.n_alpha));
  {
    dim3 grid((g.n_rows + 127) / 128, g.n_alpha);
    assemble_A_kernel<<<grid, 128, 0, s>>>(g, c->d_A);
    GRT_HIP(c, hipGetLastError());
    equilibrate_kernel<<<g.n_alpha, 256, 0, s>>>(c->d_A, g.n_rows, g.n_alpha, c->d_colscale);
    GRT_HIP(c, hipGetLastError());
  }

  // SVD of the equilibrated A (a copy: gesvd overwrites its input)
  const int m = g.n_rows, n = g.n_alpha, mn = std::min(m, n);
  cd* Awork = nullptr;
  double* Ework = nullptr;
  int* dinfo = nullptr;
  GRT_HIP(c, hipMalloc(&Awork, sizeof(cd) * nA));
  GRT_HIP(c, hipMemcpyAsync(Awork, c->d_A, sizeof(cd) * nA, hipMemcpyDeviceToDevice, s));
  GRT_HIP(c, hipMalloc(&c->d_sv, sizeof(double) * mn));
  GRT_HIP(c, hipMalloc(&c->d_U, sizeof(cd) * (size_t)m * mn));
  GRT_HIP(c, hipMalloc(&c->d_VH, sizeof(cd) * (size_t)n * n));
  GRT_HIP(c, hipMalloc(&Ework, sizeof(double) * std::max(1, mn - 1)));
  GRT_HIP(c, hipMalloc(&dinfo, sizeof(int)));
  rocblas_handle hb;
  rocblas_status rs = rocblas_create_handle(&hb);
  if (rs != rocblas_status_success) return rocblas_err(c, "rocblas_create_handle", rs);
  rocblas_set_stream(hb, s);
  rs = rocsolver_zgesvd(hb, rocblas_svect_singular, rocblas_svect_singular, m, n,
                        reinterpret_cast<rocblas_double_complex*>(Awork), m, c->d_sv,
                        reinterpret_cast<rocblas_double_complex*>(c->d_U), m,
                        reinterpret_cast<rocblas_double_complex*>(c->d_VH), n, Ework,
                        rocblas_outofplace, dinfo);
  if (rs != rocblas_status_success) {
    rocblas_destroy_handle(hb);
    return rocblas_err(c, "rocsolver_zgesvd", rs);
  }
  int hinfo = 0;
  std::vector<double> sv(mn);
  GRT_HIP(c, hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  GRT_HIP(c, hipMemcpyAsync(sv.data(), c->d_sv, sizeof(double) * mn, hipMemcpyDeviceToHost, s));
  GRT_HIP(c, hipStreamSynchronize(s));
  rocblas_destroy_handle(hb);
  hipFree(Awork);
  hipFree(Ework);
  hipFree(dinfo);
  if (hinfo != 0)
    return set_err(c, GRT_EHIP, "rocsolver_zgesvd did not converge (info=" + std::to_string(hinfo) + ")");
  int rank = 0;
  for (int k = 0; k < mn; ++k)
    if (sv[k] >= c->lay.pinv_eps * sv[0] && sv[k] > 0) ++rank;
  c->rank = rank;

  // factor blocks streamed by the apply
  GRT_HIP(c, hipMalloc(&c->d_W1, sizeof(cd) * (size_t)rank * c->n_g));
  GRT_HIP(c, hipMalloc(&c->d_W2, sizeof(cd) * (size_t)c->n_b * rank));
  GRT_HIP(c, hipMalloc(&c->d_W3, sizeof(cd) * (size_t)2 * g.Nrb * rank));
  {
    dim3 g1((c->n_g + 255) / 256, rank);
    build_W1_kernel<<<g1, 256, 0, s>>>(c->d_U, m, c->d_sv, rank, c->n_g, c->d_W1);
    dim3 g2((rank + 255) / 256, c->n_b);
    build_Wv_kernel<<<g2, 256, 0, s>>>(c->d_VH, n, c->d_colscale, 0, c->n_b, rank, c->d_W2);
    if (g.te) {
      const int nmax = std::max(c->n_g, c->n_b);
      dim3 gt((nmax + 255) / 256, rank);
      te_fold_kernel<<<gt, 256, 0, s>>>(c->d_W1, rank, c->n_g, c->d_W2, c->n_b,
                                        g.col_off[CB_A2], g.N, g.fl[1], g.pv[1]);
    }
    dim3 g3((rank + 255) / 256, 2 * g.Nrb);
    build_Wv_kernel<<<g3, 256, 0, s>>>(c->d_VH, n, c->d_colscale, g.col_off[CB_C], 2 * g.Nrb, rank,
                                       c->d_W3);
    GRT_HIP(c, hipGetLastError());
  }
  GRT_HIP(c, hipMalloc(&c->d_f, sizeof(cd) * c->n_g));
  rhs_f_kernel<<<(c->n_g + 255) / 256, 256, 0, s>>>(g, g.k[0] * cos(c->inc.phi), c->n_g, c->d_f);
  GRT_HIP(c, hipGetLastError());
  GRT_HIP(c, hipStreamSynchronize(s));
  return GRT_OK;
}

// Per-problem part: Mie diagonal, normalisation, L2L table.
static grt_status build_inclusions(grt_ctx* c) {
  hipStream_t s = c->stream;
  DevGeom& g = c->g;
  if (c->M > 0) {
    GRT_HIP(c, hipMalloc(&c->d_mie, sizeof(cd) * c->n_beta));
    mie_kernel<<<(int)((c->M + 63) / 64), 64, 0, s>>>((int)c->M, c->P, g.k[1], c->d_rad, c->d_kp,
                                                      c->d_kp_im, c->d_mie, g.te, g.pv[1],
                                                      c->inc.omega);
    GRT_HIP(c, hipMalloc(&c->d_dnorm, sizeof(double) * c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_dinv, sizeof(double) * c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_xtmp, sizeof(cd) * c->n_beta));
    dnorm_kernel<<<(int)((c->M + 63) / 64), 64, 0, s>>>((int)c->M, c->P, g.k[1], c->d_rad,
                                                        c->d_dnorm, c->d_dinv);
    int L = g.Q[1] + c->P;
    GRT_HIP(c, hipMalloc(&c->d_l2l, sizeof(cd) * (size_t)c->M * (2 * L + 1)));
    l2l_table_kernel<<<(int)((c->M + 63) / 64), 64, 0, s>>>((int)c->M, L, g.k[1], c->d_cx, c->d_cy,
                                                            c->d_l2l);
    GRT_HIP(c, hipGetLastError());
    // non-circular inclusions: dense scattering-matrix blocks (sec. 4.1) in place of
    // the Mie diagonal, which then serves only the enclosing circles' normalisation
    if (has_shapes(c)) {
      grt_status st = build_scattering_blocks(c);
      if (st != GRT_OK) return st;
    }
  }
  GRT_HIP(c, hipStreamSynchronize(s));
  return GRT_OK;
}
