// Fast translation for large M: a single-level cell scheme for T x (paper sec. 4.2
// and the fast-multipole acceleration its complexity remarks name), computing the
// same operator as the dense translation up to the truncation of the cell
// expansions.
//
// The inclusion centres are binned into an nx x ny grid of cells tiling the period
// (x in [-d/2, d/2)) and the centres' y range.  A source cell B, taken on copy
// l = -1, 0, 1 (shifted by l d, phased by alpha^l), is near a target cell A when the
// two are adjacent, |ax - (bx + l nx)| <= 1 and |ay - by| <= 1; those pairs are
// translated directly, one inclusion pair at a time, and everything else goes
// through the cells' expansions of order p (|mu| <= p):
//   P2M  M_B[mu] = sum_{m in B} sum_nu G_{nu-mu}(C_B - c_m) x_m[nu]
//   M2L  L_A[n]  = sum_B sum_mu tau^{(AB)}_{mu-n} M_B[mu],
//        tau^{(AB)}_q = sum_{l: (A, B, l) far} alpha^l F_q(C_A - C_B - l d)
//   L2L  y_j[n] += sum_q G_{q-n}(c_j - C_A) L_A[q]
// with F_q(v) = H_q(k|v|) e^{iq arg v} and G_q(v) = J_q(k|v|) e^{iq arg v} (Graf's
// theorem for the outgoing shift, the multipole-to-local translation and the local
// shift).  On a uniform grid tau^{(AB)} depends only on (ax - bx, ay - by), so the
// generators form a small table built once.  The near part writes one partial result
// per neighbour slot (3 x 3), the far part one more; the combine sums them like the
// dense translation's chunk partials.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"
#include "translate.h"

namespace {

using namespace grt;

constexpr int FMM_PMAX = 127;                 // cell order: 2p + 1 <= 255 threads
constexpr int FMM_QMAX = FMM_PMAX + 40;       // |q| <= p + P in the inclusion <-> cell shifts
constexpr int FMM_THREADS = 256;
constexpr int FMM_SLOTS = 9;                  // near neighbour slots (dx, dy) in {-1,0,1}^2
constexpr int FMM_CAP = 16;                   // inclusions per pass of the shift kernels
constexpr int FMM_SPLIT = 4;                  // source-cell shares of the cell translation

__device__ __forceinline__ cd copy_weight(cd alpha, cd alpha_inv, int l) {
  return l == 0 ? cd{1.0, 0.0} : (l > 0 ? alpha : alpha_inv);
}

// Generator table: gen[e][q + 2p], q = -2p..2p, e = (dx + nx - 1)(2 ny - 1) + dy + ny - 1
// for the cell offsets dx = ax - bx, dy = ay - by; the far copies only.
__global__ void fmm_gen_kernel(int nx, int ny, double sx, double sy, int p, double k, cd alpha,
                               cd alpha_inv, cd* gen) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int ne = (2 * nx - 1) * (2 * ny - 1);
  if (e >= ne) return;
  const int dx = e / (2 * ny - 1) - (nx - 1), dy = e % (2 * ny - 1) - (ny - 1);
  const int NQ = 4 * p + 1;
  cd* row = gen + (size_t)e * NQ;
  for (int q = 0; q < NQ; ++q) row[q] = cd{0.0, 0.0};
  for (int l = -1; l <= 1; ++l) {
    if (abs(dx - l * nx) <= 1 && abs(dy) <= 1) continue;  // near: translated directly
    const double vx = (dx - l * nx) * sx, vy = dy * sy;    // C_A - C_B - l d
    const double r = sqrt(vx * vx + vy * vy), z = k * r;
    const cd e1{vx / r, vy / r};
    const cd w = copy_weight(alpha, alpha_inv, l);
    cd hp, hc;
    hankel01(z, hp, hc);
    row[2 * p] += w * hp;
    cd ep = e1;
    for (int q = 1; q <= 2 * p; ++q) {
      const cd t = hc * ep;                 // H_q e^{iq phi}
      cd tm = hc * conj(ep);                // H_{-q} e^{-iq phi} = (-1)^q H_q e^{-iq phi}
      if (q & 1) tm = -tm;
      row[2 * p + q] += w * t;
      row[2 * p - q] += w * tm;
      const cd hn = (2.0 * q / z) * hc - hp;  // upward recurrence
      hp = hc;
      hc = hn;
      ep = ep * e1;
    }
  }
}

// J_0..J_QN(k r) and e^{i theta} of v = C - c (P2M) or c - C (L2L) for up to FMM_CAP
// inclusions of a cell at once, one thread each (Miller's recurrence is serial).
__device__ __forceinline__ void shift_rows(const int* __restrict__ order, int base, int cnt,
                                           const double* __restrict__ cx,
                                           const double* __restrict__ cy, double Cx, double Cy,
                                           double sgn, double k, int QN,
                                           double (*jn)[FMM_QMAX + 1], cd* e1s) {
  const int t = threadIdx.x;
  if (t < cnt) {
    const int m = order[base + t];
    const double vx = sgn * (Cx - cx[m]), vy = sgn * (Cy - cy[m]);
    const double r = sqrt(vx * vx + vy * vy);
    bessel_jn_array(k * r, QN, jn[t]);
    e1s[t] = r > 0 ? cd{vx / r, vy / r} : cd{1.0, 0.0};
  }
}

// acc += sum_{i = 0..len-1} G_{q0 + i} c[i], G_q = J_q e^{iq theta} from the row (J_{-q} =
// (-1)^q J_q), the phase carried along q by one product per term.
__device__ __forceinline__ void shift_dot(cd& acc, const double* jn, cd e, int q0, int len,
                                          const cd* c) {
  cd ph = q0 >= 0 ? cpowi(e, q0) : cpowi(conj(e), -q0);
  int q = q0;
  for (int i = 0; i < len; ++i, ++q) {
    const int aq = q < 0 ? -q : q;
    const double jv = (q < 0 && (aq & 1)) ? -jn[aq] : jn[aq];
    cmac(acc, jv * ph, c[i]);
    ph = ph * e;
  }
}

// P2M: one block per cell, thread t <-> mu = t - p, FMM_CAP inclusions per pass:
// M_B[mu] = sum_m sum_nu G_{nu-mu}(C_B - c_m) x_m[nu].
template <int P>
__global__ void __launch_bounds__(FMM_THREADS) fmm_p2m_kernel(
    const int* __restrict__ start, const int* __restrict__ order, const double* __restrict__ cx,
    const double* __restrict__ cy, const cd* __restrict__ x, int ny, double x0, double y0,
    double sx, double sy, int p, double k, cd* Mc) {
  constexpr int NB = 2 * P + 1;
  __shared__ double jn[FMM_CAP][FMM_QMAX + 1];
  __shared__ cd e1s[FMM_CAP];
  __shared__ cd xs[FMM_CAP * NB];
  const int cell = blockIdx.x, t = threadIdx.x;
  const double Cx = x0 + (cell / ny + 0.5) * sx, Cy = y0 + (cell % ny + 0.5) * sy;
  const int QN = P + p;
  cd acc{0.0, 0.0};
  const int e0 = start[cell], e1 = start[cell + 1];
  for (int base = e0; base < e1; base += FMM_CAP) {
    const int cnt = min(FMM_CAP, e1 - base);
    __syncthreads();  // the previous pass's rows are no longer read
    shift_rows(order, base, cnt, cx, cy, Cx, Cy, 1.0, k, QN, jn, e1s);
    for (int i = t; i < cnt * NB; i += blockDim.x)
      xs[i] = x[(size_t)order[base + i / NB] * NB + i % NB];
    __syncthreads();
    if (t < 2 * p + 1) {
      const int mu = t - p;
      for (int i = 0; i < cnt; ++i) shift_dot(acc, jn[i], e1s[i], -P - mu, NB, xs + i * NB);
    }
  }
  if (t < 2 * p + 1) Mc[(size_t)cell * (2 * p + 1) + t] = acc;
}

// M2L: block (target cell, share s of the source cells).  A thread holds FMM_RT
// consecutive outputs n and keeps a sliding window of FMM_RT generator entries
// tau_{mu - n}, so each generator load and each coefficient read from LDS serve
// FMM_RT products; the block's threads form G = FMM_THREADS / NR groups (NR threads
// cover the 2p + 1 outputs), group g taking every G-th source cell of the share, and
// the groups' sums are added through LDS in group order; partial s of L_A is written.
constexpr int FMM_RT = 4;
static_assert(FMM_RT == 4, "the window is written out for four outputs");
__global__ void __launch_bounds__(FMM_THREADS) fmm_m2l_kernel(const cd* __restrict__ Mc,
                                                             const cd* __restrict__ gen, int nx,
                                                             int ny, int p, cd* Lpart) {
  // G * NB <= FMM_RT * FMM_THREADS source coefficients, and as many partial sums
  __shared__ cd ms[FMM_RT * FMM_THREADS];
  const int A = blockIdx.x, share = blockIdx.y, t = threadIdx.x;
  const int ax = A / ny, ay = A % ny;
  const int NB = 2 * p + 1, NQ = 4 * p + 1;
  const int NR = (NB + FMM_RT - 1) / FMM_RT, G = FMM_THREADS / NR;
  const int grp = t / NR, o = (t - grp * NR) * FMM_RT;  // outputs o .. o + FMM_RT - 1
  const int ncell = nx * ny;
  const int per = (ncell + FMM_SPLIT - 1) / FMM_SPLIT;
  const int b0 = share * per, b1 = min(ncell, b0 + per);
  cd acc[FMM_RT];
#pragma unroll
  for (int u = 0; u < FMM_RT; ++u) acc[u] = cd{0.0, 0.0};
  for (int B0 = b0; B0 < b1; B0 += G) {
    const int cnt = min(G, b1 - B0);
    __syncthreads();
    for (int i = t; i < cnt * NB; i += blockDim.x) ms[i] = Mc[(size_t)B0 * NB + i];
    __syncthreads();
    if (grp < cnt) {
      const int B = B0 + grp;
      const int e = (ax - B / ny + nx - 1) * (2 * ny - 1) + (ay - B % ny + ny - 1);
      const cd* gb = gen + (size_t)e * NQ + 2 * p;  // tau_q = gb[q], |q| <= 2p
      const cd* m = ms + grp * NB;
      // w[u] = tau_{i - (o + u)}: the coefficient of output o + u times M_B[i]; the
      // padding outputs (o + u >= NB) reach q < -2p, read as zero
      cd w[FMM_RT];  // the window before i = 0
      w[0] = (-1 - o >= -2 * p) ? gb[-1 - o] : cd{0.0, 0.0};
      w[1] = (-2 - o >= -2 * p) ? gb[-2 - o] : cd{0.0, 0.0};
      w[2] = (-3 - o >= -2 * p) ? gb[-3 - o] : cd{0.0, 0.0};
      w[3] = cd{0.0, 0.0};
      for (int i = 0; i < NB; ++i) {
        w[3] = w[2];
        w[2] = w[1];
        w[1] = w[0];
        w[0] = (i - o >= -2 * p) ? gb[i - o] : cd{0.0, 0.0};
        const cd mi = m[i];
#pragma unroll
        for (int u = 0; u < FMM_RT; ++u) cmac(acc[u], w[u], mi);
      }
    }
  }
  __syncthreads();
  if (grp < G) {
#pragma unroll
    for (int u = 0; u < FMM_RT; ++u) ms[grp * NR * FMM_RT + o + u] = acc[u];
  }
  __syncthreads();
  for (int n = t; n < NB; n += blockDim.x) {
    cd s{0.0, 0.0};
    for (int g = 0; g < G; ++g) s += ms[g * NR * FMM_RT + n];
    Lpart[((size_t)share * ncell + A) * NB + n] = s;
  }
}

// L2L: one block per cell, FMM_CAP inclusions per pass, one thread per (inclusion, n):
// out[j][n] = sum_q G_{q-n}(c_j - C_A) L_A[q], L_A the sum of the FMM_SPLIT partials.
template <int P>
__global__ void __launch_bounds__(FMM_THREADS) fmm_l2l_kernel(
    const int* __restrict__ start, const int* __restrict__ order, const double* __restrict__ cx,
    const double* __restrict__ cy, const cd* __restrict__ Lpart, int ncell, int ny, double x0,
    double y0, double sx, double sy, int p, double k, cd* out) {
  constexpr int NB = 2 * P + 1;
  __shared__ double jn[FMM_CAP][FMM_QMAX + 1];
  __shared__ cd e1s[FMM_CAP];
  __shared__ cd ls[2 * FMM_PMAX + 1];
  const int cell = blockIdx.x, t = threadIdx.x;
  const double Cx = x0 + (cell / ny + 0.5) * sx, Cy = y0 + (cell % ny + 0.5) * sy;
  const int QN = P + p, NL = 2 * p + 1;
  for (int i = t; i < NL; i += blockDim.x) {
    cd v{0.0, 0.0};
    for (int s = 0; s < FMM_SPLIT; ++s) v += Lpart[((size_t)s * ncell + cell) * NL + i];
    ls[i] = v;
  }
  const int e0 = start[cell], e1 = start[cell + 1];
  for (int base = e0; base < e1; base += FMM_CAP) {
    const int cnt = min(FMM_CAP, e1 - base);
    __syncthreads();  // ls written / the previous pass's rows no longer read
    shift_rows(order, base, cnt, cx, cy, Cx, Cy, -1.0, k, QN, jn, e1s);
    __syncthreads();
    for (int it = t; it < cnt * NB; it += blockDim.x) {
      const int i = it / NB, n = it % NB - P;
      cd acc{0.0, 0.0};
      shift_dot(acc, jn[i], e1s[i], -p - n, NL, ls);
      out[(size_t)order[base + i] * NB + n + P] = acc;
    }
  }
}

// One copy of one source: acc[n] += w sum_nu F_{nu-n}(v) b[nu], v = target - source,
// F_q(v) = H_q(k|v|) e^{iq arg v} (H_0, H_1 from the table, the upward recurrence and
// powers of e^{i arg v}), in the same order of operations as the dense kernels' pair
// routine restricted to one copy.
template <int P>
__device__ __forceinline__ void copy_accumulate(cd* acc, const cd* b, double vx, double vy,
                                                double k, cd w, const double* tab) {
  constexpr int NQB = (2 * P + M2L_QB - 1) / M2L_QB;
  const double r = sqrt(vx * vx + vy * vy);
  const double z = k * r;
  const double ir = 1.0 / r;
  const cd cc{vx * ir, vy * ir};
  cd cq = cc;
  const double rz2 = 2.0 / z;
  cd h0, h1;
  hankel01_tab(z, tab, h0, h1);
  cd hp = w * h0, hc = w * h1;
#pragma unroll
  for (int n = 0; n < 2 * P + 1; ++n) cmac(acc[n], hp, b[n]);
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    cd tp[M2L_QB], tm[M2L_QB];
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      cd sp{0.0, 0.0}, sm{0.0, 0.0};
      if (q <= 2 * P) {
        sp.r = fma(hc.r, cq.r, sp.r);
        sp.r = fma(-hc.i, cq.i, sp.r);
        sp.i = fma(hc.r, cq.i, sp.i);
        sp.i = fma(hc.i, cq.r, sp.i);
        sm.r = fma(hc.r, cq.r, sm.r);
        sm.r = fma(hc.i, cq.i, sm.r);
        sm.i = fma(hc.i, cq.r, sm.i);
        sm.i = fma(-hc.r, cq.i, sm.i);
        if (q & 1) sm = -sm;
        if (q < 2 * P) {
          const cd hn = (q * rz2) * hc - hp;
          hp = hc;
          hc = hn;
          cq = cq * cc;
        }
      }
      tp[u] = sp;
      tm[u] = sm;
    }
    contract_block<P, cd, const cd*>(acc, b, qb, tp, tm);
  }
}

// Near part: one wave per (target cell, row of neighbour cells dy, group of up to 21
// of the cell's targets); lane = (target, column dx) for the 63 lanes, so the three
// source cells of the row are taken side by side.  Slot s = (dx + 1) 3 + (dy + 1) takes
// the source cell at (ax + dx, ay + dy) (x wrapping onto the copies l = -1, +1); the
// pair (j, j, 0) is excluded.  Each lane loops over its own source cell (the source
// coefficients are read from memory, lane by lane) and writes partial s + 1 of its
// target (zero for a slot outside the grid).
constexpr int FMM_NEAR_T = 21;  // targets per wave: 3 columns x 21 = 63 lanes
template <int P>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 8))) fmm_near_kernel(
    const int2* __restrict__ groups, const int* __restrict__ start, const int* __restrict__ order,
    const double* __restrict__ cx, const double* __restrict__ cy, const cd* __restrict__ x,
    int nx, int ny, double d, double k, cd alpha, cd alpha_inv, const double* __restrict__ htab,
    cd* part, int64_t n_beta) {
  constexpr int NB = 2 * P + 1;
  __shared__ double stab[HTAB_SIZE];
  for (int i = threadIdx.x; i < HTAB_SIZE; i += blockDim.x) stab[i] = htab[i];
  __syncthreads();
  const int2 gr = groups[blockIdx.x];  // (cell, offset into its list * 4 + row)
  const int A = gr.x, row = gr.y & 3, off = gr.y >> 2;
  const int ti = threadIdx.x / 3, col = threadIdx.x % 3;
  const int e = start[A] + off + ti;
  const bool live = threadIdx.x < 3 * FMM_NEAR_T && ti < FMM_NEAR_T && e < start[A + 1];
  if (!live) return;  // no barrier below
  const int j = order[e];
  const int slot = col * 3 + row;
  const int sdx = col - 1, sdy = row - 1;
  int bx = A / ny + sdx, l = 0;
  if (bx < 0) { bx += nx; l = -1; }
  if (bx >= nx) { bx -= nx; l = 1; }
  const int by = A % ny + sdy;
  cd acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = cd{0.0, 0.0};
  if (by >= 0 && by < ny) {
    const int B = bx * ny + by;
    const cd w = copy_weight(alpha, alpha_inv, l);
    // at P = 20 the one-copy routine's accumulators end up in scratch memory: use the
    // dense kernels' pair routine there, generating its middle copy only
    const cd wl[3] = {cd{0.0, 0.0}, w, cd{0.0, 0.0}};
    const double tx = cx[j], ty = cy[j];
    for (int f = start[B]; f < start[B + 1]; ++f) {
      const int m = order[f];
      if (m == j && l == 0) continue;
      const cd* b = x + (size_t)m * NB;
      if constexpr (P > 15)
        pair_accumulate<P, cd, const cd*, const double*, 0, 2 * P + 1, true>(
            acc, b, tx - (cx[m] + l * d), ty - cy[m], k, d, wl, false, false,
            (const double*)stab, 0.0);
      else
        copy_accumulate<P>(acc, b, tx - (cx[m] + l * d), ty - cy[m], k, w, (const double*)stab);
    }
  }
  cd* o = part + (size_t)(slot + 1) * n_beta + (size_t)j * NB;
#pragma unroll
  for (int n = 0; n < NB; ++n) o[n] = acc[n];
}

template <int P>
void launch_fmm(grt_ctx* c, const cd* x, hipStream_t s) {
  const int ncell = c->fmm_nx * c->fmm_ny;
  fmm_p2m_kernel<P><<<ncell, FMM_THREADS, 0, s>>>(c->d_fmm_start, c->d_fmm_order, c->d_cx,
                                                  c->d_cy, x, c->fmm_ny, c->fmm_x0, c->fmm_y0,
                                                  c->fmm_sx, c->fmm_sy, c->fmm_p, c->g.k[1],
                                                  c->d_fmm_M);
  fmm_m2l_kernel<<<dim3(ncell, FMM_SPLIT), FMM_THREADS, 0, s>>>(
      c->d_fmm_M, c->d_fmm_gen, c->fmm_nx, c->fmm_ny, c->fmm_p, c->d_fmm_L);
  fmm_l2l_kernel<P><<<ncell, FMM_THREADS, 0, s>>>(c->d_fmm_start, c->d_fmm_order, c->d_cx,
                                                  c->d_cy, c->d_fmm_L, ncell, c->fmm_ny,
                                                  c->fmm_x0, c->fmm_y0, c->fmm_sx, c->fmm_sy,
                                                  c->fmm_p, c->g.k[1], c->d_pT);
  fmm_near_kernel<P><<<(unsigned)c->fmm_ngroups, 64, 0, s>>>(c->d_fmm_groups, c->d_fmm_start, c->d_fmm_order,
                                         c->d_cx, c->d_cy, x, c->fmm_nx, c->fmm_ny, c->g.d,
                                         c->g.k[1], c->g.alpha, c->g.alpha_inv, c->d_htab,
                                         c->d_pT, c->n_beta);
}

void free_fmm(grt_ctx* c) {
  for (void* q : {(void*)c->d_fmm_start, (void*)c->d_fmm_order, (void*)c->d_fmm_groups,
                  (void*)c->d_fmm_gen, (void*)c->d_fmm_M, (void*)c->d_fmm_L})
    if (q) hipFree(q);
  c->d_fmm_start = c->d_fmm_order = nullptr;
  c->d_fmm_groups = nullptr;
  c->d_fmm_gen = c->d_fmm_M = c->d_fmm_L = nullptr;
  c->fmm_on = false;
}

}  // namespace

int fmm_partials() { return 1 + FMM_SLOTS; }

void fmm_release(grt_ctx* c) { free_fmm(c); }

grt_status fmm_apply(grt_ctx* c, const cd* x, hipStream_t s) {
  switch (c->P) {
    case 1: launch_fmm<1>(c, x, s); break;
    case 2: launch_fmm<2>(c, x, s); break;
    case 3: launch_fmm<3>(c, x, s); break;
    case 4: launch_fmm<4>(c, x, s); break;
    case 5: launch_fmm<5>(c, x, s); break;
    case 6: launch_fmm<6>(c, x, s); break;
    case 8: launch_fmm<8>(c, x, s); break;
    case 10: launch_fmm<10>(c, x, s); break;
    case 12: launch_fmm<12>(c, x, s); break;
    case 15: launch_fmm<15>(c, x, s); break;
    case 20: launch_fmm<20>(c, x, s); break;
    default: return set_err(c, GRT_EUNSUP, "the cell translation takes P <= 20");
  }
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

grt_status fmm_setup(grt_ctx* c, int p_cell, int per_cell) {
  free_fmm(c);
  const int64_t M = c->M;
  if (M == 0) return GRT_OK;
  if (c->P > 20) return set_err(c, GRT_EUNSUP, "the cell translation takes P <= 20");
  if (per_cell > 4096) return set_err(c, GRT_EINVAL, "per_cell must be at most 4096");
  const double d = c->g.d, k = c->g.k[1];
  double ymin = c->hy[0], ymax = c->hy[0];
  for (int64_t m = 1; m < M; ++m) {
    ymin = std::min(ymin, c->hy[m]);
    ymax = std::max(ymax, c->hy[m]);
  }
  const double pad = 1e-9 * (1.0 + std::fabs(ymin) + std::fabs(ymax));
  const double H = (ymax - ymin) + 2 * pad;
  if (per_cell <= 0) {
    // at least 16 inclusions per cell, and cells no narrower than k s sqrt(2) = 13: with
    // smaller k s the order k s sqrt(2) + 25 no longer holds 1e-12 per order (measured:
    // 2.4e-13 at k s sqrt(2) = 13.6, M = 10000; 6.4e-10 at 7.7, M = 30000)
    const double s_min = 13.0 / (k * std::sqrt(2.0));
    const double need = (double)M * s_min * s_min / (d * std::max(H, 1e-3 * d));
    per_cell = (int)std::min(4096.0, std::max(16.0, std::ceil(need)));
  }
  // square cells (a far pair of cells is then at least two sides apart while the two
  // half-diagonals add to 1.41 sides), about per_cell inclusions each, at least 3
  // across the period (so that a cell and its neighbours on the copies l = -1, 0, 1
  // stay distinct); the grid is centred on the centres' y range
  const double ncell_want = std::max(1.0, (double)M / per_cell);
  const double s_want = std::sqrt(d * std::max(H, 1e-3 * d) / ncell_want);
  const int nx = std::max(3, (int)std::lround(d / s_want));
  const double sx = d / nx, sy = sx;
  const int ny = std::max(1, (int)std::ceil(H / sx - 1e-9));
  const double y0 = 0.5 * (ymin + ymax) - 0.5 * ny * sy;
  // a target disk must stay inside the convergence region of its cell's local
  // expansion: radius + half-diagonal + half-diagonal < two sides
  const double rmax = *std::max_element(c->hr.begin(), c->hr.end());
  if (rmax >= 0.5 * sx)
    return set_err(c, GRT_EUNSUP, "inclusions too large for the cells: raise per_cell");
  // order of the cell expansions: k times the cell diagonal plus 25 (the measured
  // truncation error is then near 1e-13 relative on the preconditioned operator)
  int p = p_cell > 0 ? p_cell : (int)std::ceil(k * std::sqrt(sx * sx + sy * sy) + 25.0);
  if (p > FMM_PMAX)
    return set_err(c, GRT_EUNSUP, "cell expansion order above 127: use fewer inclusions per cell");
  if ((int64_t)nx * ny > 65536) return set_err(c, GRT_EUNSUP, "more than 65536 cells");
  // the generators reach H_{2p}(z) at z = k 2 s (the closest far offset, two sides):
  // keep its size, about (2p - 1)! (2 / z)^{2p} / pi, well inside FP64
  {
    const double z = 2.0 * k * sx, q = 2.0 * p;
    if (std::lgamma(q) + q * std::log(2.0 / z) - std::log(M_PI) > 600.0)
      return set_err(c, GRT_EUNSUP, "cell order too high for the cell size (generator overflow)");
  }
  // bin the centres (counting sort, stable)
  const int ncell = nx * ny;
  std::vector<int> cell(M), start(ncell + 1, 0), order(M);
  for (int64_t m = 0; m < M; ++m) {
    int ix = (int)std::floor((c->hx[m] + 0.5 * d) / sx);
    int iy = (int)std::floor((c->hy[m] - y0) / sy);
    ix = std::min(nx - 1, std::max(0, ix));
    iy = std::min(ny - 1, std::max(0, iy));
    cell[m] = ix * ny + iy;
    ++start[cell[m] + 1];
  }
  for (int i = 0; i < ncell; ++i) start[i + 1] += start[i];
  {
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int64_t m = 0; m < M; ++m) order[fill[cell[m]]++] = (int)m;
  }
  // near groups: (cell, offset * 4 + row of neighbour cells), FMM_NEAR_T targets each
  std::vector<int2> groups;
  for (int i = 0; i < ncell; ++i)
    for (int o = 0; o < start[i + 1] - start[i]; o += FMM_NEAR_T)
      for (int row = 0; row < 3; ++row) groups.push_back(int2{i, o * 4 + row});
  const int tch = 1 + FMM_SLOTS;
  if (c->m2l_nchunks_cap < tch) {  // room for the near slots' partials
    if (c->d_pT) hipFree(c->d_pT);
    c->d_pT = nullptr;
    GRT_HIP(c, hipMalloc(&c->d_pT, sizeof(cd) * (size_t)tch * c->n_beta));
    c->m2l_nchunks_cap = tch;
  }
  GRT_HIP(c, hipMalloc(&c->d_fmm_start, sizeof(int) * (ncell + 1)));
  GRT_HIP(c, hipMalloc(&c->d_fmm_order, sizeof(int) * M));
  GRT_HIP(c, hipMalloc(&c->d_fmm_groups, sizeof(int2) * groups.size()));
  const size_t ne = (size_t)(2 * nx - 1) * (2 * ny - 1);
  GRT_HIP(c, hipMalloc(&c->d_fmm_gen, sizeof(cd) * ne * (4 * p + 1)));
  GRT_HIP(c, hipMalloc(&c->d_fmm_M, sizeof(cd) * (size_t)ncell * (2 * p + 1)));
  GRT_HIP(c, hipMalloc(&c->d_fmm_L, sizeof(cd) * (size_t)FMM_SPLIT * ncell * (2 * p + 1)));
  GRT_HIP(c, hipMemcpyAsync(c->d_fmm_start, start.data(), sizeof(int) * (ncell + 1),
                            hipMemcpyHostToDevice, c->stream));
  GRT_HIP(c, hipMemcpyAsync(c->d_fmm_order, order.data(), sizeof(int) * M, hipMemcpyHostToDevice,
                            c->stream));
  GRT_HIP(c, hipMemcpyAsync(c->d_fmm_groups, groups.data(), sizeof(int2) * groups.size(),
                            hipMemcpyHostToDevice, c->stream));
  fmm_gen_kernel<<<(unsigned)((ne + 63) / 64), 64, 0, c->stream>>>(
      nx, ny, sx, sy, p, k, c->g.alpha, c->g.alpha_inv, c->d_fmm_gen);
  GRT_HIP(c, hipGetLastError());
  GRT_HIP(c, hipStreamSynchronize(c->stream));  // the host vectors above are temporaries
  c->fmm_nx = nx;
  c->fmm_ny = ny;
  c->fmm_p = p;
  c->fmm_sx = sx;
  c->fmm_sy = sy;
  c->fmm_x0 = -0.5 * d;
  c->fmm_y0 = y0;
  c->fmm_ngroups = (int)groups.size();
  c->fmm_on = true;
  return GRT_OK;
}
