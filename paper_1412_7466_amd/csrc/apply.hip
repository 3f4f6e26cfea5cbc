// The apply of the reduced operator K = I - S T + S B_phys A^+ C (paper sec. 5).
//
// Kernels, in launch order:
//  m2l_kernel<P>     alpha^T_j[n] = sum_m sum_l alpha^l sum_nu t^{(jml)}_{nu-n} x_m[nu]
//                    with t_q = H_q(k2 rho) e^{i q phi} (Graf, sec. 4.2) for the three
//                    near copies l = -1, 0, 1 (eq. repre3_mod), (j,m,l) != (j,j,0).
//                    The three copies are summed at the generator level, so one
//                    Toeplitz product is done per (j, m).  H_0, H_1 come from
//                    dev_bessel.h and H_q by upward recurrence; e^{iq phi} by powers.
//  cx_kernel         g = C x: multipole fields at the Gamma_1 / Gamma_2 nodes (value,
//                    d/dy, three copies) and at the middle walls (value, d/dx,
//                    cancelled form alpha^2 Phi(L-d) - alpha^{-1} Phi(L+2d)).
//  gemv (setup.hip)  t = Sigma^+ U^* g, w = E V t  (eq. applypA)
//  bx_kernel<P>      alpha^L_j[n] from the interface densities (P2L by Graf for H_0)
//  l2l_kernel        alpha^L_j[n] += sum_q a2_q J_{q-n}(k2 rho_j) e^{i(q-n) phi_j} (L2L)
//  combine_kernel    y = x - s o (alpha^T - alpha^L)
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

constexpr int M2L_WAVES = 4;     // waves per block: same 64 targets, sources split 4 ways
constexpr int M2L_THREADS = 64 * M2L_WAVES;
constexpr int M2L_TILE = 16;     // sources staged in LDS at a time, per wave
constexpr int M2L_QB = 4;        // generator orders produced per block of the contraction

__device__ __forceinline__ void cmac(cf& acc, cf a, cf b) {
  acc.r = fmaf(a.r, b.r, acc.r);
  acc.r = fmaf(-a.i, b.i, acc.r);
  acc.i = fmaf(a.r, b.i, acc.i);
  acc.i = fmaf(a.i, b.r, acc.i);
}
__device__ __forceinline__ cd to_acc(cd v, cd*) { return v; }
__device__ __forceinline__ cf to_acc(cd v, cf*) { return cf{(float)v.r, (float)v.i}; }

// Contribution of one source inclusion (and its copies l = -1, 0, 1) to the incoming
// coefficients acc[n] of one target, n = -P..P at index n + P:
//   acc[n] += sum_nu tau_{nu-n} x[nu],  tau_q = sum_l alpha^l H_q(k rho_l) e^{i q phi_l},
//   rho_l e^{i phi_l} = (dx - l d) + i dy  (Graf's theorem for each copy).
// The generator is FP64 (H_0, H_1 from the table, upward recurrence, powers of
// e^{i phi}) and is produced M2L_QB orders at a time; T is the accumulation type
// (cd: FP64, cf: FP32 with FP32 accumulation).  Each x[nu] is read once per block of
// orders and feeds up to 2 M2L_QB complex FMAs.  skip0 drops the copy l = 0 (the
// excluded self term); dead drops everything.  With zsafe > 0 the pair is dropped
// too when a kept copy has k rho < zsafe (left to the FP64 near-pair pass).
template <int P, typename T, typename BP, typename TabPtr>
__device__ __forceinline__ void pair_accumulate(T* acc, BP b, double dx, double dy, double k,
                                                double d, const cd* wl, bool skip0, bool dead,
                                                TabPtr tab, double zsafe) {
  constexpr int NB = 2 * P + 1;
  constexpr int NQB = (2 * P + M2L_QB - 1) / M2L_QB;
  cd hp[3], hc[3], cc[3], cq[3];
  double rz2[3];
  double zz[3];
  bool near = false;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    double ex = dx - (l - 1) * d;
    bool off = (skip0 && l == 1) || dead;
    double r = sqrt(ex * ex + dy * dy);
    if (off) r = 1.0;
    double z = k * r;
    zz[l] = z;
    if (!off && z < zsafe) near = true;
    double ir = 1.0 / r;
    cc[l] = cd{ex * ir, dy * ir};
    cq[l] = cc[l];
    rz2[l] = 2.0 / z;
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    bool off = (skip0 && l == 1) || dead || near;
    cd h0, h1;
    hankel01_tab(zz[l], tab, h0, h1);
    cd w = off ? cd{0.0, 0.0} : wl[l];
    hp[l] = w * h0;
    hc[l] = w * h1;
  }
  {
    T t0 = to_acc(hp[0] + hp[1] + hp[2], (T*)nullptr);
#pragma unroll
    for (int n = 0; n < NB; ++n) cmac(acc[n], t0, b[n]);
  }
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    T tp[M2L_QB], tm[M2L_QB];
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      cd sp{0.0, 0.0}, sm{0.0, 0.0};
      if (q <= 2 * P) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          double ac = hc[l].r * cq[l].r, bd = hc[l].i * cq[l].i;
          double ad = hc[l].r * cq[l].i, bc = hc[l].i * cq[l].r;
          sp.r += ac - bd;
          sp.i += ad + bc;
          sm.r += ac + bd;
          sm.i += bc - ad;
        }
        if (q & 1) sm = -sm;  // H_{-q} = (-1)^q H_q
        if (q < 2 * P) {
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            cd hn = (q * rz2[l]) * hc[l] - hp[l];
            hp[l] = hc[l];
            hc[l] = hn;
            cq[l] = cq[l] * cc[l];
          }
        }
      }
      tp[u] = to_acc(sp, (T*)nullptr);
      tm[u] = to_acc(sm, (T*)nullptr);
    }
    // x may be re-read here: keeps x[nu] out of registers across blocks of orders
    asm volatile("" ::: "memory");
#pragma unroll
    for (int nu = 0; nu < NB; ++nu) {
      bool need = false;
#pragma unroll
      for (int u = 0; u < M2L_QB; ++u) {
        const int q = 1 + qb * M2L_QB + u;
        if (q <= 2 * P && (nu - q >= 0 || nu + q < NB)) need = true;
      }
      if (!need) continue;
      const T bv = b[nu];
#pragma unroll
      for (int u = 0; u < M2L_QB; ++u) {
        const int q = 1 + qb * M2L_QB + u;
        if (q > 2 * P) continue;
        if (nu - q >= 0) cmac(acc[nu - q], tp[u], bv);   // acc[n] += t_q x[n+q]
        if (nu + q < NB) cmac(acc[nu + q], tm[u], bv);   // acc[n] += t_{-q} x[n-q]
      }
    }
  }
}

// Translation of the outgoing coefficients of sources [m0, m1) (and of their
// copies l = -1, 0, 1) into incoming coefficients at 64 targets (one per lane);
// the block's four waves take a quarter of the sources each, stage them in LDS
// (every lane then reads the same address: a broadcast) and are summed through
// LDS at the end.  T = cd: FP64; T = cf: FP32 contraction and accumulation with
// pairs closer than zsafe left out.
template <int P, typename T>
__global__ void __launch_bounds__(M2L_THREADS) m2l_kernel(const double* __restrict__ cx,
                                                          const double* __restrict__ cy,
                                                          const T* __restrict__ x, T* partial,
                                                          int M, int chunk, double k, double d,
                                                          cd alpha, cd alpha_inv,
                                                          const double* __restrict__ htab,
                                                          double zsafe) {
  constexpr int NB = 2 * P + 1;
  constexpr int TW = sizeof(T) / sizeof(double);  // doubles per complex value (1 or 2)
  constexpr int STAGE = M2L_WAVES * M2L_TILE * (TW * NB + 2);
  constexpr int RED = TW * NB * 64;
  constexpr int BUF = STAGE > RED ? STAGE : RED;
  __shared__ double smem[BUF];
  __shared__ double stab[HTAB_SIZE];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  T* sx = reinterpret_cast<T*>(smem) + wv * M2L_TILE * NB;
  double* scx = smem + TW * M2L_WAVES * M2L_TILE * NB + wv * 2 * M2L_TILE;
  double* scy = scx + M2L_TILE;
  const int j = blockIdx.x * 64 + lane;
  const int m0 = blockIdx.y * chunk;
  const int m1 = min(M, m0 + chunk);
  const int per = (m1 - m0 + M2L_WAVES - 1) / M2L_WAVES;
  const int s0 = m0 + wv * per;
  const int s1 = min(m1, s0 + per);
  const int ntile = (per + M2L_TILE - 1) / M2L_TILE;  // same for every wave: barriers match
  for (int t = threadIdx.x; t < HTAB_SIZE; t += M2L_THREADS) stab[t] = htab[t];
  const bool live = j < M;
  const double xj = live ? cx[j] : 0.0, yj = live ? cy[j] : 0.0;
  T acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = T{0, 0};
  const cd wl[3] = {alpha_inv, cd{1.0, 0.0}, alpha};
  for (int it = 0; it < ntile; ++it) {
    const int ts = s0 + it * M2L_TILE;
    const int cnt = max(0, min(M2L_TILE, s1 - ts));
    __syncthreads();
    for (int t = lane; t < cnt * NB; t += 64) sx[t] = x[(size_t)ts * NB + t];
    for (int t = lane; t < cnt; t += 64) {
      scx[t] = cx[ts + t];
      scy[t] = cy[ts + t];
    }
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      const int m = ts + mm;
      pair_accumulate<P, T>(acc, sx + mm * NB, xj - scx[mm], yj - scy[mm], k, d, wl, j == m,
                            !live, stab, zsafe);
    }
  }
  // sum the four waves' partial results through LDS: wave 3, then 2, then 1 add into
  // the buffer in turn, wave 0 adds its own and stores
  T* red = reinterpret_cast<T*>(smem);
  for (int src = M2L_WAVES - 1; src >= 1; --src) {
    __syncthreads();
    if (wv == src) {
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        T v = acc[n];
        if (src != M2L_WAVES - 1) {
          T o = red[n * 64 + lane];
          v.r += o.r;
          v.i += o.i;
        }
        red[n * 64 + lane] = v;
      }
    }
  }
  __syncthreads();
  if (wv == 0 && live) {
    T* out = partial + ((size_t)blockIdx.y * M + j) * NB;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      T o = red[n * 64 + lane];
      out[n] = T{acc[n].r + o.r, acc[n].i + o.i};
    }
  }
}

// FP64 translation over the near-pair lists (CSR by target): the pairs the FP32
// pass leaves out.  One lane per target; x is read from global memory.
template <int P>
__global__ void __launch_bounds__(64) m2l_near_kernel(const double* __restrict__ cx,
                                                      const double* __restrict__ cy,
                                                      const cd* __restrict__ x,
                                                      const int* __restrict__ noff,
                                                      const int* __restrict__ nlist, cd* out,
                                                      int M, double k, double d, cd alpha,
                                                      cd alpha_inv,
                                                      const double* __restrict__ htab) {
  constexpr int NB = 2 * P + 1;
  __shared__ double stab[HTAB_SIZE];
  for (int t = threadIdx.x; t < HTAB_SIZE; t += 64) stab[t] = htab[t];
  __syncthreads();
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= M) return;
  const double xj = cx[j], yj = cy[j];
  cd acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = cd{0.0, 0.0};
  const cd wl[3] = {alpha_inv, cd{1.0, 0.0}, alpha};
  for (int e = noff[j]; e < noff[j + 1]; ++e) {
    const int m = nlist[e];
    pair_accumulate<P, cd>(acc, x + (size_t)m * NB, xj - cx[m], yj - cy[m], k, d, wl, j == m,
                           false, stab, 0.0);
  }
  cd* o = out + (size_t)j * NB;
#pragma unroll
  for (int n = 0; n < NB; ++n) o[n] = acc[n];
}

constexpr int CX_TILE = 32;  // inclusions staged in LDS at a time

// Field of all multipoles (and their copies) at the C targets, one per lane:
//   target t < N: Gamma_1 node, t < 2N: Gamma_2 node (value, d/dy over 3 copies),
//   t < 2N + Nw2: middle wall node (value, d/dx, cancelled two-term form
//   alpha^2 Phi(L-d) - alpha^{-1} Phi(L+2d), Phi the l = 0 field).
// With F_n = H_n(k r) e^{in theta}: value = sum x[n] F_n and, by
// (d_x +- i d_y) F_n = -+ k F_{n+-1}, d/dx = (k/2)(A - B), d/dy = (ik/2)(A + B)
// with A = sum x[n] F_{n-1}, B = sum x[n] F_{n+1}.
// partial[chunk][t][0..1] = (value, derivative) over the chunk's inclusions.
template <int P>
__global__ void __launch_bounds__(64) cx_kernel(DevGeom g, const double* __restrict__ cx,
                                                const double* __restrict__ cy,
                                                const cd* __restrict__ x, cd* partial, int chunk,
                                                const double* __restrict__ htab) {
  constexpr int NB = 2 * P + 1;
  __shared__ cd sx[CX_TILE * NB];
  __shared__ double scx[CX_TILE], scy[CX_TILE];
  __shared__ double stab[HTAB_SIZE];
  const int nt = 2 * g.N + g.Nw[1];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int m0 = blockIdx.y * chunk;
  const int m1 = min(g.M, m0 + chunk);
  for (int i = threadIdx.x; i < HTAB_SIZE; i += 64) stab[i] = htab[i];
  const bool live = t < nt;
  const int tt = live ? t : 0;
  double tx[3], ty;
  cd w[3];
  const bool wall = tt >= 2 * g.N;
  if (!wall) {
    int i = tt % g.N;
    double x0 = -0.5 * g.d + (i + 0.5) * g.hs;
    ty = (tt < g.N) ? g.h : -g.h;
    // copies of the source at x_m + l d are equivalent to targets at x - l d
    tx[0] = x0 + g.d; w[0] = g.alpha_inv;  // l = -1
    tx[1] = x0;       w[1] = cd{1.0, 0.0};
    tx[2] = x0 - g.d; w[2] = g.alpha;      // l = +1
  } else {
    ty = g.yw[1][tt - 2 * g.N];
    tx[0] = -1.5 * g.d; w[0] = g.alpha * g.alpha;
    tx[1] = 1.5 * g.d;  w[1] = -g.alpha_inv;
    tx[2] = 1.5 * g.d;  w[2] = cd{0.0, 0.0};  // unused
  }
  const int nimg = wall ? 2 : 3;
  const double k = g.k[1];
  cd val{0, 0}, A{0, 0}, B{0, 0};
  for (int ts = m0; ts < m1; ts += CX_TILE) {
    const int cnt = min(CX_TILE, m1 - ts);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * NB; i += 64) sx[i] = x[(size_t)ts * NB + i];
    for (int i = threadIdx.x; i < cnt; i += 64) {
      scx[i] = cx[ts + i];
      scy[i] = cy[ts + i];
    }
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      const cd* b = sx + mm * NB;
#pragma unroll
      for (int im = 0; im < 3; ++im) {
        if (im >= nimg) break;
        double vx = tx[im] - scx[mm], vy = ty - scy[mm];
        double r = sqrt(vx * vx + vy * vy);
        double z = k * r;
        double ir = 1.0 / r;
        cd e{vx * ir, vy * ir};
        cd hprev, hcur;
        hankel01_tab(z, stab, hprev, hcur);
        cd sv{0, 0}, sa{0, 0}, sb{0, 0};
        cmac(sv, hprev, b[P]);
        if (P >= 1) {
          cmac(sa, hprev, b[P + 1]);
          cmac(sb, hprev, b[P - 1]);
        }
        cd ep = e;
        double rz2 = 2.0 / z;
#pragma unroll
        for (int mo = 1; mo <= P + 1; ++mo) {
          cd Fp = hcur * ep;                 // F_mo
          cd Fm = hcur * conj(ep);           // F_{-mo} = (-1)^mo H_mo e^{-i mo theta}
          if (mo & 1) Fm = -Fm;
          if (mo <= P) {
            cmac(sv, Fp, b[P + mo]);
            cmac(sv, Fm, b[P - mo]);
          }
          if (mo + 1 <= P) cmac(sa, Fp, b[P + mo + 1]);
          if (1 - mo >= -P) cmac(sa, Fm, b[P + 1 - mo]);
          if (mo - 1 <= P) cmac(sb, Fp, b[P + mo - 1]);
          if (-mo - 1 >= -P) cmac(sb, Fm, b[P - mo - 1]);
          if (mo <= P) {
            cd hn = (mo * rz2) * hcur - hprev;
            hprev = hcur;
            hcur = hn;
            ep = ep * e;
          }
        }
        val += w[im] * sv;
        A += w[im] * sa;
        B += w[im] * sb;
      }
    }
  }
  if (!live) return;
  cd der = wall ? (0.5 * k) * (A - B) : times_i((0.5 * k) * (A + B));
  cd* o = partial + ((size_t)blockIdx.y * nt + t) * 2;
  o[0] = val;
  o[1] = der;
}

// g (rows Gamma_1 v/n, Gamma_2 v/n, wall-2 v/d) from the chunk partials: one
// wavefront per target, lanes over chunks, fixed-order tree sum.
__global__ void __launch_bounds__(256) cx_reduce_kernel(DevGeom g, const cd* partial, int nchunks,
                                                        cd* gv) {
  const int nt = 2 * g.N + g.Nw[1];
  const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= nt) return;
  double vr = 0, vi = 0, dr = 0, di = 0;
  for (int c = lane; c < nchunks; c += 64) {
    cd v = partial[((size_t)c * nt + t) * 2];
    cd dv = partial[((size_t)c * nt + t) * 2 + 1];
    vr += v.r; vi += v.i; dr += dv.r; di += dv.i;
  }
  for (int off = 32; off > 0; off >>= 1) {
    vr += __shfl_xor(vr, off, 64);
    vi += __shfl_xor(vi, off, 64);
    dr += __shfl_xor(dr, off, 64);
    di += __shfl_xor(di, off, 64);
  }
  if (lane != 0) return;
  cd v{vr, vi}, dv{dr, di};
  const int N = g.N;
  if (t < N) {  // Gamma_1: row is u_1 - u_2, the inclusions live in layer 2
    gv[g.row_off[RB_G1V] + t] = -v;
    gv[g.row_off[RB_G1N] + t] = -dv;
  } else if (t < 2 * N) {
    gv[g.row_off[RB_G2V] + t - N] = v;
    gv[g.row_off[RB_G2N] + t - N] = dv;
  } else {
    gv[g.row_off[RB_W2V] + t - 2 * N] = v;
    gv[g.row_off[RB_W2D] + t - 2 * N] = dv;
  }
}

// Incoming coefficients at inclusion j from the interface densities (P2L, Graf's
// theorem for H_0 about c_j):
//   alpha_j[n] += (i/4) hs alpha^l [G_n sigma - (ik/2)(G_{n-1} + G_{n+1}) mu],
//   G_n = H_n(k|v|) e^{-in theta_v}, v = node copy - c_j,
// the mu term being d/dy of the sigma term (gradient identity).  Sources: 2 lines x
// N nodes x 3 copies = 6N node-copies, chunked over blockIdx.y.  Each G_m is used
// as soon as it is generated: it feeds acc[m] (sigma) and acc[m -+ 1] (mu).
template <int P>
__global__ void __launch_bounds__(64) bx_kernel(DevGeom g, const double* __restrict__ cx,
                                                const double* __restrict__ cy,
                                                const cd* __restrict__ w, cd* partial, int chunk,
                                                const double* __restrict__ htab) {
  constexpr int NB = 2 * P + 1;
  __shared__ double stab[HTAB_SIZE];
  for (int i = threadIdx.x; i < HTAB_SIZE; i += 64) stab[i] = htab[i];
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = blockIdx.y * chunk;
  const int s1 = min(6 * g.N, s0 + chunk);
  const bool live = j < g.M;
  const double xj = live ? cx[j] : 0.0, yj = live ? cy[j] : 0.0;
  const double k = g.k[1];
  cd acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = cd{0.0, 0.0};
  for (int sidx = s0; sidx < s1; ++sidx) {
    const int line = sidx / (3 * g.N);
    const int rem = sidx - line * 3 * g.N;
    const int l = rem / g.N - 1;
    const int i = rem - (l + 1) * g.N;
    const double sxp = -0.5 * g.d + (i + 0.5) * g.hs + l * g.d;
    const double syp = line == 0 ? g.h : -g.h;
    const cd mu = w[g.col_off[line == 0 ? CB_MU1 : CB_MU2] + i];
    const cd sg = w[g.col_off[line == 0 ? CB_SIG1 : CB_SIG2] + i];
    const cd ph = (l == 0) ? cd{1.0, 0.0} : (l > 0 ? g.alpha : g.alpha_inv);
    const cd pre = times_i((0.25 * g.hs) * ph);        // (i/4) hs alpha^l
    const cd csig = pre * sg;
    const cd cmu = pre * times_i((-0.5 * k) * mu);     // -(ik/2) mu (i/4) hs alpha^l
    const double vx = sxp - xj, vy = syp - yj;
    const double r = sqrt(vx * vx + vy * vy);
    const double z = k * r;
    const double ir = 1.0 / r;
    const cd e{vx * ir, vy * ir};
    const cd ec = conj(e);
    cd hprev, hcur;
    hankel01_tab(z, stab, hprev, hcur);
    // order 0: G_0 = H_0 -> acc[0] (sigma), acc[+-1] (mu)
    cmac(acc[P], csig, hprev);
    if (P >= 1) {
      cmac(acc[P + 1], cmu, hprev);
      cmac(acc[P - 1], cmu, hprev);
    }
    cd ep = ec, em = e;
    const double rz2 = 2.0 / z;
#pragma unroll
    for (int m = 1; m <= P + 1; ++m) {
      const cd Gp = hcur * ep;                                  // G_m = H_m e^{-im theta}
      const cd Gm = (m & 1) ? -(hcur * em) : hcur * em;        // G_{-m} = (-1)^m H_m e^{im theta}
      if (m <= P) {
        cmac(acc[P + m], csig, Gp);
        cmac(acc[P - m], csig, Gm);
      }
      // G_m feeds acc[m - 1] and acc[m + 1]; G_{-m} feeds acc[-m + 1] and acc[-m - 1]
      if (m - 1 <= P) cmac(acc[P + m - 1], cmu, Gp);
      if (m + 1 <= P) cmac(acc[P + m + 1], cmu, Gp);
      if (1 - m >= -P) cmac(acc[P + 1 - m], cmu, Gm);
      if (-m - 1 >= -P) cmac(acc[P - m - 1], cmu, Gm);
      if (m <= P) {
        const cd hn = (m * rz2) * hcur - hprev;
        hprev = hcur;
        hcur = hn;
        ep = ep * ec;
        em = em * e;
      }
    }
  }
  if (live) {
    cd* out = partial + ((size_t)blockIdx.y * g.M + j) * NB;
#pragma unroll
    for (int n = 0; n < NB; ++n) out[n] = acc[n];
  }
}

// L2L: out[j][n] = sum_q a2_q E_j[q - n], E_j[m] = J_m(k2 rho_j) e^{i m phi_j}.
// One block per inclusion: its E_j row and a2 are staged in LDS.
__global__ void __launch_bounds__(64) l2l_kernel(int M, int P, int Q2, const cd* __restrict__ E,
                                                 const cd* __restrict__ a2, cd* out) {
  extern __shared__ cd l2l_smem[];
  const int j = blockIdx.x;
  const int NB = 2 * P + 1;
  const int L = Q2 + P;
  cd* se = l2l_smem;               // 2L + 1
  cd* sa = l2l_smem + 2 * L + 1;   // 2 Q2 + 1
  const cd* e = E + (size_t)j * (2 * L + 1);
  for (int i = threadIdx.x; i < 2 * L + 1; i += blockDim.x) se[i] = e[i];
  for (int i = threadIdx.x; i < 2 * Q2 + 1; i += blockDim.x) sa[i] = a2[i];
  __syncthreads();
  for (int nn = threadIdx.x; nn < NB; nn += blockDim.x) {
    const int n = nn - P;
    cd acc{0, 0};
    for (int q = -Q2; q <= Q2; ++q) cmac(acc, sa[q + Q2], se[L + q - n]);
    out[(size_t)j * NB + nn] = acc;
  }
}

// y = x - s o (sum_c pT[c] - sum_c pB[c] - pL); any of the parts may be absent.
__global__ void combine_kernel(int nbeta, const cd* x, const cd* s, const cd* pT, int nT,
                               const cd* pB, int nB, const cd* pL, cd* y, int mode) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbeta) return;
  cd t{0, 0}, b{0, 0};
  for (int c = 0; c < nT; ++c) t += pT[(size_t)c * nbeta + i];
  for (int c = 0; c < nB; ++c) b += pB[(size_t)c * nbeta + i];
  if (pL) b += pL[i];
  if (mode == 0) {  // full K
    y[i] = x[i] - s[i] * (t - b);
  } else if (mode == 1) {  // T x only
    y[i] = t;
  } else if (mode == 2) {  // B A^+ C x only
    y[i] = b;
  } else {  // rhs: s o (B part)
    y[i] = s[i] * b;
  }
}

// Event pair for timing one translation launch (when profiling is on).
hipEvent_t* prof_pair(grt_ctx* c) {
  if (!c->prof) return nullptr;
  if (c->prof_used + 2 > c->prof_ev.size()) {
    for (int t = 0; t < 64; ++t) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      c->prof_ev.push_back(e);
    }
  }
  hipEvent_t* p = &c->prof_ev[c->prof_used];
  c->prof_used += 2;
  return p;
}

template <int P>
void launch_m2l(grt_ctx* c, const cd* x) {
  dim3 grid((unsigned)((c->M + 63) / 64), c->m2l_nchunks);
  hipEvent_t* ev = prof_pair(c);
  if (ev) hipEventRecord(ev[0], c->stream);
  m2l_kernel<P, cd><<<grid, M2L_THREADS, 0, c->stream>>>(
      c->d_cx, c->d_cy, x, c->d_pT, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d, c->g.alpha,
      c->g.alpha_inv, c->d_htab, 0.0);
  if (ev) hipEventRecord(ev[1], c->stream);
}

template <int P>
void launch_m2l32(grt_ctx* c, const cf* x32) {
  dim3 grid((unsigned)((c->M + 63) / 64), c->m2l_nchunks);
  hipEvent_t* ev = prof_pair(c);
  if (ev) hipEventRecord(ev[0], c->stream);
  m2l_kernel<P, cf><<<grid, M2L_THREADS, 0, c->stream>>>(
      c->d_cx, c->d_cy, x32, c->d_pT32, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d, c->g.alpha,
      c->g.alpha_inv, c->d_htab, c->zsafe);
  if (ev) hipEventRecord(ev[1], c->stream);
}

template <int P>
void launch_near(grt_ctx* c, const cd* x) {
  m2l_near_kernel<P><<<(unsigned)((c->M + 63) / 64), 64, 0, c->stream>>>(
      c->d_cx, c->d_cy, x, c->d_noff, c->d_nlist, c->d_pN, (int)c->M, c->g.k[1], c->g.d,
      c->g.alpha, c->g.alpha_inv, c->d_htab);
}

__global__ void to_f32_kernel(const cd* x, cf* y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = cf{(float)x[i].r, (float)x[i].i};
}

// y = x - s o ((sum_c pT32[c] + pN) - sum_c pB[c] - pL): the mixed-precision apply.
__global__ void combine_mixed_kernel(int nbeta, const cd* x, const cd* s, const cf* pT, int nT,
                                     const cd* pN, const cd* pB, int nB, const cd* pL, cd* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbeta) return;
  cd t = pN[i];
  for (int c = 0; c < nT; ++c) {
    cf v = pT[(size_t)c * nbeta + i];
    t.r += v.r;
    t.i += v.i;
  }
  cd b = pL[i];
  for (int c = 0; c < nB; ++c) b += pB[(size_t)c * nbeta + i];
  y[i] = x[i] - s[i] * (t - b);
}

// Near-pair lists: pairs (j, m) with some kept copy at k rho < zsafe.
__device__ bool near_pair(const double* cx, const double* cy, int j, int m, double k, double d,
                          double zsafe) {
  for (int l = -1; l <= 1; ++l) {
    if (j == m && l == 0) continue;
    double dx = cx[j] - cx[m] - l * d, dy = cy[j] - cy[m];
    if (k * sqrt(dx * dx + dy * dy) < zsafe) return true;
  }
  return false;
}

__global__ void near_count_kernel(const double* cx, const double* cy, int M, double k, double d,
                                  double zsafe, int* cnt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int c = 0;
  for (int m = 0; m < M; ++m) c += near_pair(cx, cy, j, m, k, d, zsafe);
  cnt[j] = c;
}

// exclusive prefix sum of cnt[0..M) into off[0..M] (one thread; setup only)
__global__ void near_scan_kernel(const int* cnt, int M, int* off) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int s = 0;
  for (int j = 0; j < M; ++j) {
    off[j] = s;
    s += cnt[j];
  }
  off[M] = s;
}

__global__ void near_fill_kernel(const double* cx, const double* cy, int M, double k, double d,
                                 double zsafe, const int* off, int* list) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int p = off[j];
  for (int m = 0; m < M; ++m)
    if (near_pair(cx, cy, j, m, k, d, zsafe)) list[p++] = m;
}

template <int P>
void launch_cx(grt_ctx* c, const cd* x) {
  const int nt = 2 * c->g.N + c->g.Nw[1];
  dim3 grid((nt + 63) / 64, c->c_nchunks);
  cx_kernel<P><<<grid, 64, 0, c->stream>>>(c->g, c->d_cx, c->d_cy, x, c->d_pC, c->c_chunk,
                                            c->d_htab);
}

template <int P>
void launch_bx(grt_ctx* c, const cd* w) {
  dim3 grid((unsigned)((c->M + 63) / 64), c->b_nchunks);
  bx_kernel<P><<<grid, 64, 0, c->stream>>>(c->g, c->d_cx, c->d_cy, w, c->d_pB, c->b_chunk,
                                           c->d_htab);
}

#define GRT_P_DISPATCH(FN, P, ...)                        \
  switch (P) {                                            \
    case 1: FN<1>(__VA_ARGS__); break;                    \
    case 2: FN<2>(__VA_ARGS__); break;                    \
    case 3: FN<3>(__VA_ARGS__); break;                    \
    case 4: FN<4>(__VA_ARGS__); break;                    \
    case 5: FN<5>(__VA_ARGS__); break;                    \
    case 6: FN<6>(__VA_ARGS__); break;                    \
    case 8: FN<8>(__VA_ARGS__); break;                    \
    case 10: FN<10>(__VA_ARGS__); break;                  \
    case 12: FN<12>(__VA_ARGS__); break;                  \
    case 15: FN<15>(__VA_ARGS__); break;                  \
    case 20: FN<20>(__VA_ARGS__); break;                  \
    default: return set_err(c, GRT_EUNSUP, "multipole order P not compiled in"); \
  }

}  // namespace

bool supported_P(int P) {
  switch (P) {
    case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 15: case 20:
      return true;
    default:
      return false;
  }
}

grt_status apply_alloc(grt_ctx* c) {
  const int64_t M = c->M;
  // vectors of the low-rank path: also needed without inclusions (Bragg amplitudes)
  GRT_HIP(c, hipMalloc(&c->d_gvec, sizeof(cd) * (size_t)c->n_g));
  GRT_HIP(c, hipMalloc(&c->d_tvec, sizeof(cd) * (size_t)std::max(1, c->rank)));
  GRT_HIP(c, hipMalloc(&c->d_wvec, sizeof(cd) * (size_t)c->n_b));
  if (M == 0) return GRT_OK;
  // Work split: every kernel gets enough (target tile, source chunk) blocks to
  // give each of the 1024 SIMDs about two waves; partial sums per chunk are
  // added in a fixed order afterwards (deterministic results).
  auto split = [](int64_t nsrc, int64_t tiles, int64_t want_waves, int64_t min_chunk,
                  int& chunk, int& nchunks) {
    int64_t nc = std::max<int64_t>(1, (want_waves + tiles - 1) / tiles);
    nc = std::min<int64_t>(nc, std::max<int64_t>(1, (nsrc + min_chunk - 1) / min_chunk));
    int64_t ch = (nsrc + nc - 1) / nc;
    chunk = (int)ch;
    nchunks = (int)((nsrc + ch - 1) / ch);
  };
  const int nt = 2 * c->g.N + c->g.Nw[1];
  split(M, (M + 63) / 64, 2048 / M2L_WAVES, 4 * M2L_WAVES, c->m2l_chunk, c->m2l_nchunks);
  split(M, (nt + 63) / 64, 2048, 4, c->c_chunk, c->c_nchunks);
  split(6 * (int64_t)c->g.N, (M + 63) / 64, 1024, 16, c->b_chunk, c->b_nchunks);
  GRT_HIP(c, hipMalloc(&c->d_pT, sizeof(cd) * (size_t)c->m2l_nchunks * c->n_beta));
  GRT_HIP(c, hipMalloc(&c->d_pC, sizeof(cd) * (size_t)c->c_nchunks * nt * 2));
  GRT_HIP(c, hipMalloc(&c->d_pB, sizeof(cd) * (size_t)c->b_nchunks * c->n_beta));
  GRT_HIP(c, hipMalloc(&c->d_pL, sizeof(cd) * (size_t)c->n_beta));
  // mixed-precision path: FP32 copy of x, FP32 partials, near-pair lists and results.
  // zsafe: the smallest k2*rho with (2P-1)! (2/z)^{2P} / pi <= 1e30, the large-order
  // size of |H_{2P}(z)|, so that every FP32 generator value and product stays finite.
  {
    const int q = 2 * c->P;
    c->zsafe = 1.1 * 2.0 * std::exp((std::lgamma((double)q) - std::log(M_PI * 1e30)) / q);
    GRT_HIP(c, hipMalloc(&c->d_x32, sizeof(cf) * (size_t)c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_pT32, sizeof(cf) * (size_t)c->m2l_nchunks * c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_pN, sizeof(cd) * (size_t)c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_noff, sizeof(int) * (size_t)(M + 1)));
    int* cnt = nullptr;
    GRT_HIP(c, hipMalloc(&cnt, sizeof(int) * (size_t)M));
    const unsigned nbk = (unsigned)((M + 127) / 128);
    near_count_kernel<<<nbk, 128, 0, c->stream>>>(c->d_cx, c->d_cy, (int)M, c->g.k[1], c->g.d,
                                                   c->zsafe, cnt);
    near_scan_kernel<<<1, 64, 0, c->stream>>>(cnt, (int)M, c->d_noff);
    int total = 0;
    GRT_HIP(c, hipMemcpyAsync(&total, c->d_noff + M, sizeof(int), hipMemcpyDeviceToHost,
                              c->stream));
    GRT_HIP(c, hipStreamSynchronize(c->stream));
    c->n_near = total;
    GRT_HIP(c, hipMalloc(&c->d_nlist, sizeof(int) * (size_t)std::max(1, total)));
    near_fill_kernel<<<nbk, 128, 0, c->stream>>>(c->d_cx, c->d_cy, (int)M, c->g.k[1], c->g.d,
                                                  c->zsafe, c->d_noff, c->d_nlist);
    GRT_HIP(c, hipGetLastError());
    GRT_HIP(c, hipStreamSynchronize(c->stream));
    hipFree(cnt);
  }
  return GRT_OK;
}

// w = A^+ g on the prefix entries B reads, then alpha^L into pB (partials) and pL.
static grt_status lowrank_tail(grt_ctx* c, const cd* gvec) {
  hipStream_t s = c->stream;
  launch_gemv_rows(s, c->d_W1, gvec, c->d_tvec, c->rank, c->n_g);
  launch_gemv_rows(s, c->d_W2, c->d_tvec, c->d_wvec, c->n_b, c->rank);
  GRT_P_DISPATCH(launch_bx, c->P, c, c->d_wvec);
  {
    const int L = c->g.Q[1] + c->P;
    size_t sh = sizeof(cd) * (size_t)(2 * L + 1 + 2 * c->g.Q[1] + 1);
    l2l_kernel<<<(unsigned)c->M, 64, sh, s>>>((int)c->M, c->P, c->g.Q[1], c->d_l2l,
                                             c->d_wvec + c->g.col_off[CB_A2], c->d_pL);
  }
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

static grt_status cx_apply(grt_ctx* c, const cd* x) {
  const int nt = 2 * c->g.N + c->g.Nw[1];
  GRT_P_DISPATCH(launch_cx, c->P, c, x);
  cx_reduce_kernel<<<(nt + 3) / 4, 256, 0, c->stream>>>(c->g, c->d_pC, c->c_nchunks, c->d_gvec);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

static grt_status run_apply(grt_ctx* c, const cd* x, cd* y, int mode) {
  if (c->M == 0) return GRT_OK;
  hipStream_t s = c->stream;
  bool needT = (mode == 0 || mode == 1);
  bool needB = (mode == 0 || mode == 2);
  if (needT) GRT_P_DISPATCH(launch_m2l, c->P, c, x);
  if (needB) {
    grt_status st = cx_apply(c, x);
    if (st != GRT_OK) return st;
    st = lowrank_tail(c, c->d_gvec);
    if (st != GRT_OK) return st;
  }
  int n = (int)c->n_beta;
  combine_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, x, c->d_mie, c->d_pT, needT ? c->m2l_nchunks : 0,
                                                 c->d_pB, needB ? c->b_nchunks : 0,
                                                 needB ? c->d_pL : nullptr, y, mode);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

grt_status apply_K(grt_ctx* c, const cd* x, cd* y) { return run_apply(c, x, y, 0); }

// K32 x: FP32 translation between well-separated pairs, FP64 for near pairs, the
// layer correction and the preconditioner.
grt_status apply_K_mixed(grt_ctx* c, const cd* x, cd* y) {
  if (c->M == 0) return GRT_OK;
  hipStream_t s = c->stream;
  const int n = (int)c->n_beta;
  to_f32_kernel<<<(n + 255) / 256, 256, 0, s>>>(x, c->d_x32, n);
  GRT_P_DISPATCH(launch_m2l32, c->P, c, c->d_x32);
  GRT_P_DISPATCH(launch_near, c->P, c, x);
  grt_status st = cx_apply(c, x);
  if (st != GRT_OK) return st;
  st = lowrank_tail(c, c->d_gvec);
  if (st != GRT_OK) return st;
  combine_mixed_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, x, c->d_mie, c->d_pT32, c->m2l_nchunks,
                                                       c->d_pN, c->d_pB, c->b_nchunks, c->d_pL,
                                                       y);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}
grt_status apply_T_only(grt_ctx* c, const cd* x, cd* y) { return run_apply(c, x, y, 1); }
grt_status apply_lowrank_only(grt_ctx* c, const cd* x, cd* y) { return run_apply(c, x, y, 2); }

grt_status rhs_b(grt_ctx* c, cd* b) {
  if (c->M == 0) return GRT_OK;
  grt_status st = lowrank_tail(c, c->d_f);
  if (st != GRT_OK) return st;
  int n = (int)c->n_beta;
  combine_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(n, nullptr, c->d_mie, nullptr, 0, c->d_pB,
                                                         c->b_nchunks, c->d_pL, b, 3);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

__global__ void sub_kernel(int n, const cd* a, const cd* b, cd* o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] - (b ? b[i] : cd{0, 0});
}

// c and d blocks of alpha = A^+ (f - C beta) into out[0 .. 2 Nrb).
grt_status bragg_alpha(grt_ctx* c, const cd* beta, cd* out) {
  hipStream_t s = c->stream;
  if (c->M > 0) {
    grt_status st = cx_apply(c, beta);
    if (st != GRT_OK) return st;
  }
  // g = f - C beta (prefix rows; both vanish elsewhere)
  sub_kernel<<<(c->n_g + 255) / 256, 256, 0, s>>>(c->n_g, c->d_f, c->M > 0 ? c->d_gvec : nullptr,
                                                   c->d_gvec);
  launch_gemv_rows(s, c->d_W1, c->d_gvec, c->d_tvec, c->rank, c->n_g);
  launch_gemv_rows(s, c->d_W3, c->d_tvec, out, 2 * c->g.Nrb, c->rank);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}
