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
#include <mutex>
#include <string>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"
#include "translate.h"

namespace {

using namespace grt;

template <int P, typename T>
__global__ void __launch_bounds__(M2L_THREADS) m2l_kernel(const double* __restrict__ cx,
                                                          const double* __restrict__ cy,
                                                          const T* __restrict__ x, T* partial,
                                                          int M, int chunk, double k, double d,
                                                          cd alpha, cd alpha_inv,
                                                          const double* __restrict__ htab,
                                                          double zsafe) {
  m2l_block<P, T>(cx, cy, x, partial, M, chunk, k, d, alpha, alpha_inv, htab, zsafe, blockIdx.x,
                  blockIdx.y);
}

// Outputs [LO, LO + NH) only (index n + P): the on-the-fly translation split over two
// launches, each recomputing the generator, so that a lane holds half the
// accumulators (FP64) and two waves fit on a SIMD.
template <int P, int LO, int NH>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(M2L_HALF_MINW, 8))) m2l_half_kernel(const double* __restrict__ cx,
                                                               const double* __restrict__ cy,
                                                               const cd* __restrict__ x,
                                                               cd* partial, int M, int chunk,
                                                               double k, double d, cd alpha,
                                                               cd alpha_inv,
                                                               const double* __restrict__ htab) {
  m2l_block<P, cd, LO, NH>(cx, cy, x, partial, M, chunk, k, d, alpha, alpha_inv, htab, 0.0,
                           blockIdx.x, blockIdx.y);
}

template <int P>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(P <= 15 ? 2 : 1, 8))) m2l_table_kernel(const cd* __restrict__ table,
                                                                const cd* __restrict__ x,
                                                                cd* partial, int M, int Mpad,
                                                                int chunk) {
  m2l_table_block<P>(table, x, partial, M, Mpad, chunk, blockIdx.x, blockIdx.y);
}

template <int P>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(P <= 15 ? 3 : 1, 8))) m2l_table2_kernel(const cd* __restrict__ table,
                                                                 const cd* __restrict__ x,
                                                                 cd* partial, int M, int Mpad,
                                                                 int chunk) {
  m2l_table2_block<P>(table, x, partial, M, Mpad, chunk, blockIdx.x, blockIdx.y);
}

// FP32 translation of the well-separated pairs from the resident FP32 table
template <int P>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(3, 8))) m2l_table32_kernel(const cf* __restrict__ table,
                                                                  const cf* __restrict__ x,
                                                                  cf* partial, int M, int Mpad,
                                                                  int chunk) {
  m2l_table_block<P, cf>(table, x, partial, M, Mpad, chunk, blockIdx.x, blockIdx.y);
}

template <int P>
__global__ void __launch_bounds__(64) table32_build_kernel(const double* __restrict__ cx,
                                                           const double* __restrict__ cy, int M,
                                                           int Mpad, int chunk, double k,
                                                           double d, cd alpha, cd alpha_inv,
                                                           const double* __restrict__ htab,
                                                           double zsafe, cf* table) {
  table_build_block<P, cf>(cx, cy, M, Mpad, chunk, k, d, alpha, alpha_inv, htab, table,
                           blockIdx.x, blockIdx.y, zsafe);
}

template <int P>
__global__ void __launch_bounds__(64) table_build_kernel(const double* __restrict__ cx,
                                                         const double* __restrict__ cy, int M,
                                                         int Mpad, int chunk, double k, double d,
                                                         cd alpha, cd alpha_inv,
                                                         const double* __restrict__ htab,
                                                         cd* table) {
  table_build_block<P>(cx, cy, M, Mpad, chunk, k, d, alpha, alpha_inv, htab, table, blockIdx.x,
                       blockIdx.y);
}

template <int P>
__global__ void __launch_bounds__(64 * CX_WAVES) cx_kernel(DevGeom g, const double* __restrict__ cx,
                                                const double* __restrict__ cy,
                                                const cd* __restrict__ x, cd* partial, int chunk,
                                                const double* __restrict__ htab) {
  cx_block<P>(g, cx, cy, x, partial, chunk, htab, blockIdx.x, blockIdx.y);
}

template <int P>
__global__ void __launch_bounds__(64 * BX_WAVES) bx_kernel(DevGeom g, const double* __restrict__ cx,
                                                const double* __restrict__ cy,
                                                const cd* __restrict__ w, cd* partial, int chunk,
                                                const double* __restrict__ htab) {
  bx_block<P>(g, cx, cy, w, partial, chunk, htab, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) cx_reduce_rows_kernel(DevGeom g, const cd* partial,
                                                             int nchunks, cd* gv) {
  cx_reduce_rows(g, partial, nchunks, gv, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) l2l_kernel(int M, int P, int Q2, const cd* __restrict__ E,
                                                  const cd* __restrict__ a2, cd* out, int ntb) {
  l2l_block(M, P, Q2, E, a2, out, blockIdx.x, ntb);
}

// Sum of the partial results of entry i: each block takes 64 entries, its four
// waves a quarter of the chunks each, added in a fixed order through LDS.
constexpr int CMB_ENTRIES = 64;
template <typename TT>
__device__ __forceinline__ cd chunk_sum(const TT* part, int nch, size_t stride, int64_t i, int grp,
                                        bool live) {
  cd acc{0, 0};
  if (live)
    for (int c = grp; c < nch; c += 4) {
      const TT v = part[(size_t)c * stride + i];
      acc.r += v.r;
      acc.i += v.i;
    }
  return acc;
}

__device__ __forceinline__ cd group_total(cd v, cd* red, int lane, int grp) {
  red[grp * CMB_ENTRIES + lane] = v;
  __syncthreads();
  cd t = red[lane];
  for (int g2 = 1; g2 < 4; ++g2) t += red[g2 * CMB_ENTRIES + lane];
  __syncthreads();
  return t;
}

// y = x - s o (sum_c pT[c] - sum_c pB[c] - pL)   (mode 0, full K)
// y = sum_c pT[c]                                (mode 1, T x)
// y = sum_c pB[c] + pL                           (mode 2, B_phys A^+ C x, or alpha0)
// y = s o (sum_c pB[c] + pL)                     (mode 3, right-hand side)
// y = sum_c pT[c] - sum_c pB[c] - pL             (mode 4: w of y = x - S w, dense S)
// then y *= oscale when given.  Any of the parts may be absent.
__global__ void __launch_bounds__(256) combine_kernel(int nbeta, const cd* x, const cd* s,
                                                      const cd* pT, int nT, const cd* pB, int nB,
                                                      const cd* pL, cd* y, int mode,
                                                      const double* oscale) {
  __shared__ cd red[4 * CMB_ENTRIES];
  const int lane = threadIdx.x & (CMB_ENTRIES - 1), grp = threadIdx.x / CMB_ENTRIES;
  const int64_t i = (int64_t)blockIdx.x * CMB_ENTRIES + lane;
  const bool live = i < nbeta;
  const cd t = group_total(chunk_sum(pT, nT, nbeta, i, grp, live), red, lane, grp);
  cd b = group_total(chunk_sum(pB, nB, nbeta, i, grp, live), red, lane, grp);
  if (grp != 0 || !live) return;
  if (pL) b += pL[i];
  cd v;
  if (mode == 0) v = x[i] - s[i] * (t - b);
  else if (mode == 1) v = t;
  else if (mode == 2) v = b;
  else if (mode == 4) v = t - b;
  else v = s[i] * b;
  y[i] = oscale ? oscale[i] * v : v;
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
  if (c->d_table && c->table_lanes == 2) {
    dim3 grid2((unsigned)((c->M + 31) / 32), c->m2l_nchunks);
    m2l_table2_kernel<P><<<grid2, M2L_THREADS, 0, c->stream>>>(c->d_table, x, c->d_pT, (int)c->M,
                                                               c->table_mpad, c->m2l_chunk);
  } else if (c->d_table) {
    m2l_table_kernel<P><<<grid, M2L_THREADS, 0, c->stream>>>(c->d_table, x, c->d_pT, (int)c->M,
                                                             c->table_mpad, c->m2l_chunk);
  } else if (c->m2l_split == 2) {
    constexpr int NB = 2 * P + 1, H0 = (NB + 1) / 2;
    m2l_half_kernel<P, 0, H0><<<grid, M2L_THREADS, 0, c->stream>>>(
        c->d_cx, c->d_cy, x, c->d_pT, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d, c->g.alpha,
        c->g.alpha_inv, c->d_htab);
    m2l_half_kernel<P, H0, NB - H0><<<grid, M2L_THREADS, 0, c->stream>>>(
        c->d_cx, c->d_cy, x, c->d_pT, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d, c->g.alpha,
        c->g.alpha_inv, c->d_htab);
  } else
    m2l_kernel<P, cd><<<grid, M2L_THREADS, 0, c->stream>>>(
        c->d_cx, c->d_cy, x, c->d_pT, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d, c->g.alpha,
        c->g.alpha_inv, c->d_htab, 0.0);
  if (ev) hipEventRecord(ev[1], c->stream);
}

template <int P>
void launch_table_build(grt_ctx* c) {
  const int chunk = 16;
  dim3 grid((unsigned)((c->M + 63) / 64), (unsigned)((c->M + chunk - 1) / chunk));
  table_build_kernel<P><<<grid, 64, 0, c->stream>>>(c->d_cx, c->d_cy, (int)c->M, c->table_mpad,
                                                     chunk, c->g.k[1], c->g.d, c->g.alpha,
                                                     c->g.alpha_inv, c->d_htab, c->d_table);
}

template <int P>
void launch_table32_build(grt_ctx* c) {
  const int chunk = 16;
  dim3 grid((unsigned)((c->M + 63) / 64), (unsigned)((c->M + chunk - 1) / chunk));
  table32_build_kernel<P><<<grid, 64, 0, c->stream>>>(
      c->d_cx, c->d_cy, (int)c->M, c->table32_mpad, chunk, c->g.k[1], c->g.d, c->g.alpha,
      c->g.alpha_inv, c->d_htab, c->zsafe, c->d_table32);
}

template <int P>
void launch_m2l32(grt_ctx* c, const cf* x32) {
  dim3 grid((unsigned)((c->M + 63) / 64), c->m2l_nchunks);
  hipEvent_t* ev = prof_pair(c);
  if (ev) hipEventRecord(ev[0], c->stream);
  if (c->d_table32)
    m2l_table32_kernel<P><<<grid, M2L_THREADS, 0, c->stream>>>(
        c->d_table32, x32, c->d_pT32, (int)c->M, c->table32_mpad, c->m2l_chunk);
  else
    m2l_kernel<P, cf><<<grid, M2L_THREADS, 0, c->stream>>>(
        c->d_cx, c->d_cy, x32, c->d_pT32, (int)c->M, c->m2l_chunk, c->g.k[1], c->g.d,
        c->g.alpha, c->g.alpha_inv, c->d_htab, c->zsafe);
  if (ev) hipEventRecord(ev[1], c->stream);
}

template <int P>
void launch_near(grt_ctx* c, const cd* x) {
  const int np = (int)c->n_near;
  if (np > 0)
    m2l_near_kernel<P><<<(unsigned)((np + 63) / 64), 64, 0, c->stream>>>(
        c->d_cx, c->d_cy, x, c->d_ntgt, c->d_nlist, c->d_npart, np, c->g.k[1], c->g.d,
        c->g.alpha, c->g.alpha_inv, c->d_htab);
  const int tot = (int)(c->M * c->nb);
  near_reduce_kernel<<<(tot + 255) / 256, 256, 0, c->stream>>>(c->d_noff, c->d_npart, (int)c->M,
                                                               c->nb, c->d_pN);
}

__global__ void to_f32_kernel(const cd* x, cf* y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = cf{(float)x[i].r, (float)x[i].i};
}

// y = x - s o ((sum_c pT32[c] + pN) - sum_c pB[c] - pL): the mixed-precision apply.
__global__ void __launch_bounds__(256) combine_mixed_kernel(int nbeta, const cd* x, const cd* s,
                                                            const cf* pT, int nT, const cd* pN,
                                                            const cd* pB, int nB, const cd* pL,
                                                            cd* y, const double* oscale) {
  __shared__ cd red[4 * CMB_ENTRIES];
  const int lane = threadIdx.x & (CMB_ENTRIES - 1), grp = threadIdx.x / CMB_ENTRIES;
  const int64_t i = (int64_t)blockIdx.x * CMB_ENTRIES + lane;
  const bool live = i < nbeta;
  cd t = group_total(chunk_sum(pT, nT, nbeta, i, grp, live), red, lane, grp);
  cd b = group_total(chunk_sum(pB, nB, nbeta, i, grp, live), red, lane, grp);
  if (grp != 0 || !live) return;
  t += pN[i];
  b += pL[i];
  // without s: the vector w of y = x - S w (dense scattering matrices)
  const cd v = s ? x[i] - s[i] * (t - b) : t - b;
  y[i] = oscale ? oscale[i] * v : v;
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
                                 double zsafe, const int* off, int* list, int* tgt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int p = off[j];
  for (int m = 0; m < M; ++m)
    if (near_pair(cx, cy, j, m, k, d, zsafe)) {
      tgt[p] = j;
      list[p++] = m;
    }
}

template <int P>
void launch_cx(grt_ctx* c, const cd* x, hipStream_t st) {
  const int nt = 2 * c->g.N + c->g.Nw[1];
  dim3 grid((nt + 63) / 64, c->c_nchunks);
  cx_kernel<P><<<grid, 64 * CX_WAVES, 0, st>>>(c->g, c->d_cx, c->d_cy, x, c->d_pC, c->c_chunk,
                                               c->d_htab);
}

template <int P>
void launch_bx(grt_ctx* c, const cd* w, hipStream_t st) {
  dim3 grid((unsigned)((c->M + 63) / 64), c->b_nchunks);
  bx_kernel<P><<<grid, 64 * BX_WAVES, 0, st>>>(c->g, c->d_cx, c->d_cy, w, c->d_pB, c->b_chunk,
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

// Split nsrc sources into chunks so that tiles x chunks covers about want_waves
// work-groups (at least min_chunk sources per chunk).
static void split_work(int64_t nsrc, int64_t tiles, int64_t want_waves, int64_t min_chunk,
                       int& chunk, int& nchunks) {
  int64_t nc = std::max<int64_t>(1, (want_waves + tiles - 1) / tiles);
  nc = std::min<int64_t>(nc, std::max<int64_t>(1, (nsrc + min_chunk - 1) / min_chunk));
  int64_t ch = (nsrc + nc - 1) / nc;
  chunk = (int)ch;
  nchunks = (int)((nsrc + ch - 1) / ch);
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
  // added in a fixed order afterwards (deterministic results).  The translation's
  // split can be re-chosen by measurement (autotune_m2l); its partial buffers are
  // sized for the largest candidate.
  const int nt = 2 * c->g.N + c->g.Nw[1];
  split_work(M, (M + 63) / 64, 2048 / M2L_WAVES, 4 * M2L_WAVES, c->m2l_chunk, c->m2l_nchunks);
  {
    int ch, nc;
    split_work(M, (M + 63) / 64, M2L_TUNE_MAX_WAVES / M2L_WAVES, 4 * M2L_WAVES, ch, nc);
    c->m2l_nchunks_cap = std::max(nc, c->m2l_nchunks);
  }
  split_work(M, (nt + 63) / 64, 2048 / CX_WAVES, 4 * CX_WAVES, c->c_chunk, c->c_nchunks);
  split_work(2 * (int64_t)c->g.N, (M + 63) / 64, 2048 / BX_WAVES, 2 * BX_WAVES, c->b_chunk,
             c->b_nchunks);
  // the coupling launches' candidates (autotune_coupling) go down to CX_TUNE_MIN_PER
  // and BX_TUNE_MIN_PER sources per wave, within CX_TUNE_MAX_CHUNKS and
  // BX_TUNE_MAX_CHUNKS partial results (the P2L partials are n_beta entries each)
  c->c_nchunks_cap = std::max<int>(
      c->c_nchunks, (int)std::min<int64_t>(CX_TUNE_MAX_CHUNKS, (M + CX_WAVES * CX_TUNE_MIN_PER - 1) /
                                                                   (CX_WAVES * CX_TUNE_MIN_PER)));
  c->b_nchunks_cap = std::max<int>(
      c->b_nchunks,
      (int)std::min<int64_t>(BX_TUNE_MAX_CHUNKS, (2 * (int64_t)c->g.N + BX_WAVES * BX_TUNE_MIN_PER - 1) /
                                                     (BX_WAVES * BX_TUNE_MIN_PER)));
  GRT_HIP(c, hipMalloc(&c->d_pT, sizeof(cd) * (size_t)c->m2l_nchunks_cap * c->n_beta));
  GRT_HIP(c, hipMalloc(&c->d_pC, sizeof(cd) * (size_t)c->c_nchunks_cap * nt * 2));
  GRT_HIP(c, hipMalloc(&c->d_pB, sizeof(cd) * (size_t)c->b_nchunks_cap * c->n_beta));
  GRT_HIP(c, hipMalloc(&c->d_pL, sizeof(cd) * (size_t)c->n_beta));
  // mixed-precision path: FP32 copy of x, FP32 partials, near-pair lists and results.
  // zsafe: the smallest k2*rho with (2P-1)! (2/z)^{2P} / pi <= 1e30, the large-order
  // size of |H_{2P}(z)|, so that every FP32 generator value and product stays finite.
  {
    const int q = 2 * c->P;
    c->zsafe = 1.1 * 2.0 * std::exp((std::lgamma((double)q) - std::log(M_PI * 1e30)) / q);
    GRT_HIP(c, hipMalloc(&c->d_x32, sizeof(cf) * (size_t)c->n_beta));
    GRT_HIP(c, hipMalloc(&c->d_pT32, sizeof(cf) * (size_t)c->m2l_nchunks_cap * c->n_beta));
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
    GRT_HIP(c, hipMalloc(&c->d_ntgt, sizeof(int) * (size_t)std::max(1, total)));
    GRT_HIP(c, hipMalloc(&c->d_npart, sizeof(cd) * (size_t)std::max(1, total) * c->nb));
    near_fill_kernel<<<nbk, 128, 0, c->stream>>>(c->d_cx, c->d_cy, (int)M, c->g.k[1], c->g.d,
                                                  c->zsafe, c->d_noff, c->d_nlist, c->d_ntgt);
    GRT_HIP(c, hipGetLastError());
    GRT_HIP(c, hipStreamSynchronize(c->stream));
    hipFree(cnt);
  }
  return GRT_OK;
}

// w = A^+ g on the prefix entries B reads, then alpha^L into pB (partials) and pL.
static grt_status lowrank_tail(grt_ctx* c, const cd* gvec, hipStream_t s = nullptr) {
  if (!s) s = c->stream;
  launch_gemv_rows(s, c->d_W1, gvec, c->d_tvec, c->rank, c->n_g);
  launch_gemv_rows(s, c->d_W2, c->d_tvec, c->d_wvec, c->n_b, c->rank);
  GRT_P_DISPATCH(launch_bx, c->P, c, c->d_wvec, s);
  {
    const int ntb = l2l_targets_per_block(c->P, c->g.Q[1]);
    const size_t sh = l2l_lds_bytes(c->P, c->g.Q[1], ntb);
    l2l_kernel<<<(unsigned)((c->M + ntb - 1) / ntb), 64, sh, s>>>(
        (int)c->M, c->P, c->g.Q[1], c->d_l2l, c->d_wvec + c->g.col_off[CB_A2], c->d_pL, ntb);
  }
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

static grt_status cx_apply(grt_ctx* c, const cd* x, hipStream_t s = nullptr) {
  if (!s) s = c->stream;
  const int nt = 2 * c->g.N + c->g.Nw[1];
  GRT_P_DISPATCH(launch_cx, c->P, c, x, s);
  cx_reduce_rows_kernel<<<(nt + 255) / 256, 256, 0, s>>>(c->g, c->d_pC, c->c_nchunks, c->d_gvec);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

static grt_status run_apply(grt_ctx* c, const cd* x, cd* y, int mode,
                            const double* oscale = nullptr) {
  if (c->M == 0) return GRT_OK;
  hipStream_t s = c->stream;
  bool needT = (mode == 0 || mode == 1);
  bool needB = (mode == 0 || mode == 2);
  if (needT && needB && c->overlap && c->stream2) {
    // C x, A^+ and B_phys w (ALU-bound) on the second stream, concurrently with the
    // translation; the combine waits for both
    GRT_HIP(c, hipEventRecord(c->ev_fork, s));
    GRT_HIP(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
    grt_status st = cx_apply(c, x, c->stream2);
    if (st != GRT_OK) return st;
    st = lowrank_tail(c, c->d_gvec, c->stream2);
    if (st != GRT_OK) return st;
    GRT_HIP(c, hipEventRecord(c->ev_join, c->stream2));
    if (c->fmm_on) {
      st = fmm_apply(c, x, s);
      if (st != GRT_OK) return st;
    } else {
      GRT_P_DISPATCH(launch_m2l, c->P, c, x);
    }
    GRT_HIP(c, hipStreamWaitEvent(s, c->ev_join, 0));
  } else {
    if (needT && c->fmm_on) {
      grt_status st = fmm_apply(c, x, s);
      if (st != GRT_OK) return st;
    } else if (needT) {
      GRT_P_DISPATCH(launch_m2l, c->P, c, x);
    }
    if (needB) {
      grt_status st = cx_apply(c, x);
      if (st != GRT_OK) return st;
      st = lowrank_tail(c, c->d_gvec);
      if (st != GRT_OK) return st;
    }
  }
  int n = (int)c->n_beta;
  // non-circular inclusions: w = T x - B x first, then y = x - S w with the blocks
  const bool dense = c->d_sblk && mode == 0;
  const int tch = c->fmm_on ? fmm_partials() : c->m2l_nchunks;
  combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
      n, x, c->d_mie, c->d_pT, needT ? tch : 0, c->d_pB, needB ? c->b_nchunks : 0,
      needB ? c->d_pL : nullptr, dense ? c->d_wS : y, dense ? 4 : mode,
      dense ? nullptr : oscale);
  if (dense) launch_sblock_apply(c, x, c->d_wS, y, 0, oscale, s);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

grt_status apply_K(grt_ctx* c, const cd* x, cd* y, const double* oscale) {
  return run_apply(c, x, y, 0, oscale);
}

// K32 x: FP32 translation between well-separated pairs (generator on the fly, or
// from the resident FP32 table), FP64 for near pairs, the layer correction and the
// preconditioner.  With the two-stream option the FP64 layer correction runs on the
// second stream alongside the translation.
grt_status apply_K_mixed(grt_ctx* c, const cd* x, cd* y, const double* oscale) {
  if (c->fmm_on) return set_err(c, GRT_EUNSUP, "the cell translation is FP64 only");
  if (c->M == 0) return GRT_OK;
  hipStream_t s = c->stream;
  const int n = (int)c->n_beta;
  const bool ovl = c->overlap && c->stream2;
  grt_status st = GRT_OK;
  if (ovl) {
    GRT_HIP(c, hipEventRecord(c->ev_fork, s));
    GRT_HIP(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
    st = cx_apply(c, x, c->stream2);
    if (st != GRT_OK) return st;
    st = lowrank_tail(c, c->d_gvec, c->stream2);
    if (st != GRT_OK) return st;
    GRT_HIP(c, hipEventRecord(c->ev_join, c->stream2));
  }
  to_f32_kernel<<<(n + 255) / 256, 256, 0, s>>>(x, c->d_x32, n);
  GRT_P_DISPATCH(launch_m2l32, c->P, c, c->d_x32);
  GRT_P_DISPATCH(launch_near, c->P, c, x);
  if (ovl) {
    GRT_HIP(c, hipStreamWaitEvent(s, c->ev_join, 0));
  } else {
    st = cx_apply(c, x);
    if (st != GRT_OK) return st;
    st = lowrank_tail(c, c->d_gvec);
    if (st != GRT_OK) return st;
  }
  const bool dense = c->d_sblk != nullptr;
  combine_mixed_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
      n, x, dense ? nullptr : c->d_mie, c->d_pT32, c->m2l_nchunks, c->d_pN, c->d_pB,
      c->b_nchunks, c->d_pL, dense ? c->d_wS : y, dense ? nullptr : oscale);
  if (dense) launch_sblock_apply(c, x, c->d_wS, y, 0, oscale, s);
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
  const bool dense = c->d_sblk != nullptr;
  combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, c->stream>>>(
      n, nullptr, c->d_mie, nullptr, 0, c->d_pB, c->b_nchunks, c->d_pL, dense ? c->d_wS : b,
      dense ? 2 : 3, nullptr);
  if (dense) launch_sblock_apply(c, nullptr, c->d_wS, b, 1, nullptr, c->stream);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

// Resident translation table: allocate (zeroed: rows of targets >= M stay zero) and
// fill it, or free it.
size_t table_bytes(const grt_ctx* c) {
  const size_t mpad = (size_t)((c->M + 63) / 64) * 64;
  return mpad * (size_t)c->M * (size_t)(4 * c->P + 1) * sizeof(cd);
}

grt_status table_set(grt_ctx* c, bool on) {
  graph_reset(c);
  ++c->gen;
  if (c->d_table) {
    hipStreamSynchronize(c->stream);
    hipFree(c->d_table);
    c->d_table = nullptr;
  }
  if (!on || c->M == 0) return GRT_OK;
  const size_t bytes = table_bytes(c);
  size_t free_b = 0, total_b = 0;
  GRT_HIP(c, hipMemGetInfo(&free_b, &total_b));
  if (bytes + ((size_t)1 << 30) > free_b)
    return set_err(c, GRT_ENOMEM, "translation table of " + std::to_string(bytes >> 20) +
                                      " MiB does not fit in free device memory");
  c->table_mpad = (int)(((c->M + 63) / 64) * 64);
  GRT_HIP(c, hipMalloc(&c->d_table, bytes));
  GRT_HIP(c, hipMemsetAsync(c->d_table, 0, bytes, c->stream));
  GRT_P_DISPATCH(launch_table_build, c->P, c);
  GRT_HIP(c, hipGetLastError());
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  return GRT_OK;
}

// Resident FP32 table of the well-separated pairs (the mixed-precision apply's
// translation): allocate, zero and fill it, or free it.
size_t table32_bytes(const grt_ctx* c) {
  const size_t mpad = (size_t)((c->M + 63) / 64) * 64;
  return mpad * (size_t)c->M * (size_t)(4 * c->P + 1) * sizeof(cf);
}

grt_status table32_set(grt_ctx* c, bool on) {
  graph_reset(c);
  ++c->gen;
  if (c->d_table32) {
    hipStreamSynchronize(c->stream);
    hipFree(c->d_table32);
    c->d_table32 = nullptr;
  }
  if (!on || c->M == 0) return GRT_OK;
  const size_t bytes = table32_bytes(c);
  size_t free_b = 0, total_b = 0;
  GRT_HIP(c, hipMemGetInfo(&free_b, &total_b));
  if (bytes + ((size_t)1 << 30) > free_b)
    return set_err(c, GRT_ENOMEM, "FP32 translation table of " + std::to_string(bytes >> 20) +
                                      " MiB does not fit in free device memory");
  c->table32_mpad = (int)(((c->M + 63) / 64) * 64);
  GRT_HIP(c, hipMalloc(&c->d_table32, bytes));
  GRT_HIP(c, hipMemsetAsync(c->d_table32, 0, bytes, c->stream));
  GRT_P_DISPATCH(launch_table32_build, c->P, c);
  GRT_HIP(c, hipGetLastError());
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  return GRT_OK;
}

// Measure the translation launch, with the pass that adds its partial results, for
// several source-chunk counts (work-group counts from 256 to M2L_TUNE_MAX_WAVES) in
// the current mode (on the fly: also split over two launches; or resident table) and
// keep the fastest.  Reports up to cap (chunks, split, ms) triples.
grt_status autotune_m2l(grt_ctx* c, int cap, int* n_out, int* chunks_out, int* splits_out,
                        double* ms_out) {
  if (c->fmm_on) return set_err(c, GRT_EUNSUP, "autotune the dense translation (cell translation on)");
  if (c->M == 0) {
    if (n_out) *n_out = 0;
    return GRT_OK;
  }
  hipStream_t s = c->stream;
  const int64_t M = c->M;
  hipEvent_t e0, e1;
  GRT_HIP(c, hipEventCreate(&e0));
  GRT_HIP(c, hipEventCreate(&e1));
  cd* ytmp = nullptr;
  GRT_HIP(c, hipMalloc(&ytmp, sizeof(cd) * (size_t)c->n_beta));
  const bool prof = c->prof;
  c->prof = false;
  GRT_HIP(c, hipMemsetAsync(c->d_xtmp, 0, sizeof(cd) * (size_t)c->n_beta, s));
  // the variant: on the fly, one launch or two half-output launches (m2l_split);
  // with the resident table, one or two lanes per target (table_lanes)
  const bool table = c->d_table != nullptr;
  int best_chunk = c->m2l_chunk, best_n = c->m2l_nchunks,
      best_split = table ? c->table_lanes : c->m2l_split, count = 0;
  double best_ms = 1e300;
  for (int split = 1; split <= 2; ++split) {
    int last_nc = -1;
    for (int64_t waves = 256; waves <= M2L_TUNE_MAX_WAVES; waves *= 2) {
      int ch, nc;
      split_work(M, (M + 63) / 64, waves / M2L_WAVES, 4 * M2L_WAVES, ch, nc);
      if (nc == last_nc || nc > c->m2l_nchunks_cap) continue;
      last_nc = nc;
      c->m2l_chunk = ch;
      c->m2l_nchunks = nc;
      if (table)
        c->table_lanes = split;
      else
        c->m2l_split = split;
      // each candidate is timed with the pass that adds its partial results (the
      // combine reads one partial per chunk)
      const int n = (int)c->n_beta;
      for (int r = 0; r < 2; ++r) {
        GRT_P_DISPATCH(launch_m2l, c->P, c, c->d_xtmp);
        combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
            n, c->d_xtmp, c->d_mie, c->d_pT, c->m2l_nchunks, c->d_pB, 0, nullptr, ytmp, 1, nullptr);
      }
      GRT_HIP(c, hipEventRecord(e0, s));
      const int reps = 5;
      for (int r = 0; r < reps; ++r) {
        GRT_P_DISPATCH(launch_m2l, c->P, c, c->d_xtmp);
        combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
            n, c->d_xtmp, c->d_mie, c->d_pT, c->m2l_nchunks, c->d_pB, 0, nullptr, ytmp, 1, nullptr);
      }
      GRT_HIP(c, hipEventRecord(e1, s));
      GRT_HIP(c, hipEventSynchronize(e1));
      float ms = 0.f;
      GRT_HIP(c, hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / reps;
      if (count < cap) {
        if (chunks_out) chunks_out[count] = nc;
        if (splits_out) splits_out[count] = split;
        if (ms_out) ms_out[count] = per;
      }
      ++count;
      if (per < best_ms) {
        best_ms = per;
        best_chunk = ch;
        best_n = nc;
        best_split = split;
      }
    }
  }
  c->m2l_chunk = best_chunk;
  c->m2l_nchunks = best_n;
  if (table)
    c->table_lanes = best_split;
  else
    c->m2l_split = best_split;
  c->prof = prof;
  graph_reset(c);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(ytmp);
  GRT_HIP(c, hipGetLastError());
  if (n_out) *n_out = std::min(count, cap);
  return GRT_OK;
}

// Launch shapes of the coupling kernels, chosen by measurement: for each candidate
// number of sources per wave (chunk = waves per block x that number, so the waves of
// a block get equal shares) time the kernel together with the pass that adds its
// per-chunk partial results (cx_reduce for C x; the combine, which reads the P2L
// partials, for B_phys w), and keep the fastest.  Inputs are zero: the kernels' cost
// does not depend on the values.
grt_status autotune_coupling(grt_ctx* c) {
  if (c->M == 0) return GRT_OK;
  hipStream_t s = c->stream;
  const int64_t M = c->M;
  const int nt = 2 * c->g.N + c->g.Nw[1];
  const int n = (int)c->n_beta;
  cd* ytmp = nullptr;
  GRT_HIP(c, hipMalloc(&ytmp, sizeof(cd) * (size_t)n));
  hipEvent_t e0, e1;
  GRT_HIP(c, hipEventCreate(&e0));
  GRT_HIP(c, hipEventCreate(&e1));
  GRT_HIP(c, hipMemsetAsync(c->d_xtmp, 0, sizeof(cd) * (size_t)n, s));
  GRT_HIP(c, hipMemsetAsync(c->d_wvec, 0, sizeof(cd) * (size_t)c->n_b, s));
  // launch() enqueues one candidate and returns its status
  auto time_it = [&](auto&& launch) -> double {
    for (int r = 0; r < 2; ++r)
      if (launch() != GRT_OK) return -1.0;
    hipEventRecord(e0, s);
    const int reps = 6;
    for (int r = 0; r < reps; ++r) launch();
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    return ms / reps;
  };
  static const int per_wave[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 48, 64};
  {  // C x
    int best_ch = c->c_chunk, best_nc = c->c_nchunks, last = -1;
    double best = 1e300;
    for (int p : per_wave) {
      const int ch = CX_WAVES * p;
      const int nc = (int)((M + ch - 1) / ch);
      if (p < CX_TUNE_MIN_PER || nc == last || nc > c->c_nchunks_cap) continue;
      last = nc;
      c->c_chunk = ch;
      c->c_nchunks = nc;
      const double ms = time_it([&]() -> grt_status {
        GRT_P_DISPATCH(launch_cx, c->P, c, c->d_xtmp, s);
        cx_reduce_rows_kernel<<<(nt + 255) / 256, 256, 0, s>>>(c->g, c->d_pC, c->c_nchunks,
                                                               c->d_gvec);
        return GRT_OK;
      });
      if (ms < 0) break;
      if (ms < best) { best = ms; best_ch = ch; best_nc = nc; }
    }
    c->c_chunk = best_ch;
    c->c_nchunks = best_nc;
  }
  {  // B_phys w (P2L) with the combine that reads its partials
    int best_ch = c->b_chunk, best_nc = c->b_nchunks, last = -1;
    double best = 1e300;
    const int64_t ns = 2 * (int64_t)c->g.N;
    for (int p : per_wave) {
      const int ch = BX_WAVES * p;
      const int nc = (int)((ns + ch - 1) / ch);
      if (p < BX_TUNE_MIN_PER || nc == last || nc > c->b_nchunks_cap) continue;
      last = nc;
      c->b_chunk = ch;
      c->b_nchunks = nc;
      const double ms = time_it([&]() -> grt_status {
        GRT_P_DISPATCH(launch_bx, c->P, c, c->d_wvec, s);
        combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
            n, c->d_xtmp, c->d_mie, c->d_pT, 0, c->d_pB, c->b_nchunks, c->d_pL, ytmp, 2, nullptr);
        return GRT_OK;
      });
      if (ms < 0) break;
      if (ms < best) { best = ms; best_ch = ch; best_nc = nc; }
    }
    c->b_chunk = best_ch;
    c->b_nchunks = best_nc;
  }
  graph_reset(c);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(ytmp);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

// alpha0 = B_phys A^+ f: the incoming coefficients the layered structure alone sends
// to every inclusion (the right-hand side before the Mie diagonal).
grt_status incident_alpha(grt_ctx* c, cd* out) {
  if (c->M == 0) return GRT_OK;
  grt_status st = lowrank_tail(c, c->d_f);
  if (st != GRT_OK) return st;
  int n = (int)c->n_beta;
  combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, c->stream>>>(
      n, nullptr, c->d_mie, nullptr, 0, c->d_pB, c->b_nchunks, c->d_pL, out, 2, nullptr);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

__global__ void sub_kernel(int n, const cd* a, const cd* b, cd* o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] - (b ? b[i] : cd{0, 0});
}

// Every entry of alpha = A^+ (f - C beta): t = W1 g, alpha = (E V) t with E V built
// into W for all n_alpha entries.
grt_status alpha_full(grt_ctx* c, const cd* beta, cd* out, cd* W) {
  hipStream_t s = c->stream;
  if (c->M > 0) {
    grt_status st = cx_apply(c, beta);
    if (st != GRT_OK) return st;
  }
  sub_kernel<<<(c->n_g + 255) / 256, 256, 0, s>>>(c->n_g, c->d_f, c->M > 0 ? c->d_gvec : nullptr,
                                                   c->d_gvec);
  launch_gemv_rows(s, c->d_W1, c->d_gvec, c->d_tvec, c->rank, c->n_g);
  launch_build_Wv(s, c, 0, c->g.n_alpha, W);
  launch_gemv_rows(s, W, c->d_tvec, out, c->g.n_alpha, c->rank);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
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

// ---------------------------------------------------------------------------
// y = T x without a context and without any allocation by the call.  The per-chunk
// partial sums of the translation go to `scratch`, a file-scope device array of
// fixed size, and the H_0 / H_1 table to `noalloc_htab`; both exist on every device
// the library runs on for the life of the process.  Host code never passes the
// arrays' names to a kernel (on the host they are stand-ins, not device addresses):
// the first call on a device looks up their device addresses there with
// hipGetSymbolAddress and keeps them per device.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static __device__ __align__(256) double noalloc_htab[HTAB_SIZE];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocDevice {
  cd* scratch = nullptr;
  double* htab = nullptr;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Device addresses of this device's arrays; on the first call on the device also
// fills its H_0 / H_1 table (a synchronous copy of host-built coefficients).
grt_status noalloc_device(int dev, hipStream_t s, NoallocDevice& out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  NoallocDevice& nd = g_noalloc[dev];
  if (nd.scratch) {
    out = nd;
    return GRT_OK;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return GRT_EHIP;
  if (cap != hipStreamCaptureStatusNone) return GRT_ESTATE;  // first call must not be captured
  void* ps = nullptr;
  void* ph = nullptr;
  if (hipGetSymbolAddress(&ps, HIP_SYMBOL(scratch)) != hipSuccess || !ps) return GRT_EHIP;
  if (hipGetSymbolAddress(&ph, HIP_SYMBOL(noalloc_htab)) != hipSuccess || !ph) return GRT_EHIP;
  std::vector<double> tab(HTAB_SIZE);
  for (int k = 0; k < HTAB_NI; ++k) htab_interval(k, tab.data() + (size_t)k * HTAB_STRIDE);
  if (hipMemcpy(ph, tab.data(), sizeof(double) * HTAB_SIZE, hipMemcpyHostToDevice) != hipSuccess)
    return GRT_EHIP;
  nd.scratch = static_cast<cd*>(ps);
  nd.htab = static_cast<double*>(ph);
  out = nd;
  return GRT_OK;
}

template <int P>
void launch_m2l_noalloc(hipStream_t s, const double* cx, const double* cy, const cd* x, cd* part,
                        int M, int chunk, int nchunks, double k, double d, cd alpha,
                        const double* htab) {
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)nchunks);
  const cd alpha_inv{alpha.r, -alpha.i};  // |alpha| = 1
  m2l_kernel<P, cd><<<grid, M2L_THREADS, 0, s>>>(cx, cy, x, part, M, chunk, k, d, alpha,
                                                  alpha_inv, htab, 0.0);
}

#define GRT_P_DISPATCH_NOCTX(FN, P, ...)                \
  switch (P) {                                          \
    case 1: FN<1>(__VA_ARGS__); break;                  \
    case 2: FN<2>(__VA_ARGS__); break;                  \
    case 3: FN<3>(__VA_ARGS__); break;                  \
    case 4: FN<4>(__VA_ARGS__); break;                  \
    case 5: FN<5>(__VA_ARGS__); break;                  \
    case 6: FN<6>(__VA_ARGS__); break;                  \
    case 8: FN<8>(__VA_ARGS__); break;                  \
    case 10: FN<10>(__VA_ARGS__); break;                \
    case 12: FN<12>(__VA_ARGS__); break;                \
    case 15: FN<15>(__VA_ARGS__); break;                \
    case 20: FN<20>(__VA_ARGS__); break;                \
    default: return GRT_EUNSUP;                         \
  }

}  // namespace

extern "C" grt_status grt_apply_T_noalloc(int64_t M, int P, double k2, double d, double alpha_re,
                                          double alpha_im, const double* cx_dev,
                                          const double* cy_dev, const void* x_dev, void* y_dev,
                                          void* hip_stream) {
  if (M < 1 || M > (int64_t)1 << 30 || P < 1 || !(k2 > 0) || !(d > 0) || !cx_dev || !cy_dev ||
      !x_dev || !y_dev || x_dev == y_dev || !std::isfinite(alpha_re) || !std::isfinite(alpha_im) ||
      std::fabs(std::hypot(alpha_re, alpha_im) - 1.0) > 1e-12)
    return GRT_EINVAL;
  if (!supported_P(P)) return GRT_EUNSUP;
  const int64_t nbeta = M * (2 * P + 1);
  const int64_t max_chunks = (int64_t)(NOALLOC_SCRATCH_BYTES / (sizeof(cd) * (size_t)nbeta));
  if (max_chunks < 1) return GRT_EINVAL;  // one partial result does not fit
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return GRT_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  NoallocDevice nd;
  grt_status st = noalloc_device(dev, s, nd);
  if (st != GRT_OK) return st;
  // the default launch shape of the context path, limited by what the scratch holds
  int chunk = 0, nchunks = 0;
  split_work(M, (M + 63) / 64, 2048 / M2L_WAVES, 4 * M2L_WAVES, chunk, nchunks);
  if (nchunks > max_chunks) {
    chunk = (int)((M + max_chunks - 1) / max_chunks);
    nchunks = (int)((M + chunk - 1) / chunk);
  }
  const cd* x = static_cast<const cd*>(x_dev);
  cd* y = static_cast<cd*>(y_dev);
  GRT_P_DISPATCH_NOCTX(launch_m2l_noalloc, P, s, cx_dev, cy_dev, x, nd.scratch, (int)M, chunk,
                       nchunks, k2, d, cd{alpha_re, alpha_im}, nd.htab);
  const int n = (int)nbeta;
  combine_kernel<<<(n + CMB_ENTRIES - 1) / CMB_ENTRIES, 256, 0, s>>>(
      n, nullptr, nullptr, nd.scratch, nchunks, nullptr, 0, nullptr, y, 1, nullptr);
  if (hipGetLastError() != hipSuccess) return GRT_EHIP;
  return GRT_OK;
}
