// Batched solves: many problems (geometries of uneven M, angles, frequencies) solved
// together, each step of GMRES advancing all of them with one launch per kernel.
//
// Layout: the coefficient vectors of all problems are concatenated, problem i
// occupying segments [seg0_i, seg0_i + nseg_i) of SEG entries (zero padded), so that
// every elementwise and reduction kernel runs once over the whole batch and finds
// its problem through a segment -> problem table.  The apply kernels run over lists
// of work items (problem, block x, block y) built once per batch; each item runs
// the same block-level code as a single-problem launch (translate.h), with the
// problem's descriptor in device memory.  Problems are grouped by multipole order
// P (a compile-time parameter of the translation code).
//
// The Krylov method is the single-problem one (restarted GMRES, CGS2, Givens, on
// the normalised operator D K D^{-1}), run in lockstep: every problem has its own
// Hessenberg matrix, rotations and residual; a problem that has converged keeps its
// own step count k_i and takes no further updates.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "translate.h"

using namespace grt;

namespace {

constexpr int SEG = 1024;   // entries per segment (256 threads x 4)
constexpr int BT = 256;

struct InstDesc {
  DevGeom g;
  const double *cx, *cy, *htab;
  const cd *mie, *W1, *W2, *l2l, *f;
  int M, P, nb, rank, n_g, n_b, Q2;
  int m2l_chunk, m2l_nchunks, c_chunk, c_nchunks, b_chunk, b_nchunks;
  cd *pT, *pC, *pB, *pL, *gvec, *tvec, *wvec;
  int64_t off, nbeta;
  int seg0, nseg;
  // mixed precision (GRT_FP32): FP32 partials of the well-separated pairs, near-pair
  // CSR lists with their FP64 per-pair results and sums (the problem's own buffers)
  cf* pT32;
  cd *npart, *pN;
  const int *noff, *nlist, *ntgt;
  int n_near;
  double zsafe;
  // resident translation table of the FP64 apply (null: generator on the fly)
  const cd* table;
  int mpad;
  // resident FP32 table of the well-separated pairs (mixed apply; null: on the fly)
  const cf* table32;
  int mpad32;
  // non-circular inclusions: dense scattering-matrix blocks [M][2P+1][2P+1] and the
  // problem's w vector of y = x - S w (null: the Mie diagonal)
  const cd* sblk;
  cd* wS;
  int split;  // 2: FP64 on-the-fly translation as two half-output launches
  // 0 once the lockstep solver has no further use for this problem's applies: every
  // apply kernel then skips its work items and the combine writes zeros
  int active;
};

struct Item {
  int inst, x, y;
};

// ---------------------------------------------------------------------------
// batched apply kernels
// ---------------------------------------------------------------------------

template <int P>
__global__ void __launch_bounds__(M2L_THREADS) m2l_batched(const InstDesc* __restrict__ D,
                                                           const Item* __restrict__ it,
                                                           const cd* __restrict__ X) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  m2l_block<P, cd>(q.cx, q.cy, X + q.off, q.pT, q.M, q.m2l_chunk, q.g.k[1], q.g.d, q.g.alpha,
                   q.g.alpha_inv, q.htab, 0.0, w.x, w.y);
}

template <int P>
__global__ void __launch_bounds__(64 * CX_WAVES) cx_batched(const InstDesc* __restrict__ D,
                                                 const Item* __restrict__ it,
                                                 const cd* __restrict__ X) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  cx_block<P>(q.g, q.cx, q.cy, X + q.off, q.pC, q.c_chunk, q.htab, w.x, w.y);
}

// FP64 translation on the fly, outputs [LO, LO + NH) only (the split launch shape)
template <int P, int LO, int NH>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(M2L_HALF_MINW, 8)))
m2lh_batched(const InstDesc* __restrict__ D, const Item* __restrict__ it,
             const cd* __restrict__ X) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  m2l_block<P, cd, LO, NH>(q.cx, q.cy, X + q.off, q.pT, q.M, q.m2l_chunk, q.g.k[1], q.g.d,
                           q.g.alpha, q.g.alpha_inv, q.htab, 0.0, w.x, w.y);
}

// FP64 translation from the problem's resident table
template <int P>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(P <= 15 ? 2 : 1, 8)))
m2lt_batched(const InstDesc* __restrict__ D, const Item* __restrict__ it,
             const cd* __restrict__ X) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  m2l_table_block<P>(q.table, X + q.off, q.pT, q.M, q.mpad, q.m2l_chunk, w.x, w.y);
}

// FP32 translation of the well-separated pairs (near pairs, k2 rho < zsafe, skipped)
template <int P>
__global__ void __launch_bounds__(M2L_THREADS) m2l32_batched(const InstDesc* __restrict__ D,
                                                             const Item* __restrict__ it,
                                                             const cf* __restrict__ X32) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  m2l_block<P, cf>(q.cx, q.cy, X32 + q.off, q.pT32, q.M, q.m2l_chunk, q.g.k[1], q.g.d, q.g.alpha,
                   q.g.alpha_inv, q.htab, q.zsafe, w.x, w.y);
}

// FP32 translation of the well-separated pairs from the problem's FP32 table
template <int P>
__global__ void __launch_bounds__(M2L_THREADS) __attribute__((amdgpu_waves_per_eu(3, 8))) m2lt32_batched(const InstDesc* __restrict__ D,
                                                              const Item* __restrict__ it,
                                                              const cf* __restrict__ X32) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  m2l_table_block<P, cf>(q.table32, X32 + q.off, q.pT32, q.M, q.mpad32, q.m2l_chunk, w.x, w.y);
}

// the near pairs [64 x, 64 x + 64) of a problem in FP64, one lane per pair
template <int P>
__global__ void __launch_bounds__(64) near_batched(const InstDesc* __restrict__ D,
                                                   const Item* __restrict__ it,
                                                   const cd* __restrict__ X) {
  __shared__ double stab[HTAB_SIZE];
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  for (int t = threadIdx.x; t < HTAB_SIZE; t += 64) stab[t] = q.htab[t];
  __syncthreads();
  const int e = w.x * 64 + threadIdx.x;
  if (e < q.n_near)
    near_pair<P>(q.cx, q.cy, X + q.off, q.ntgt, q.nlist, q.npart, e, q.g.k[1], q.g.d, q.g.alpha,
                 q.g.alpha_inv, stab);
}

// per-target sums of the near-pair results, entries [256 x, 256 x + 256) of a problem
__global__ void __launch_bounds__(256) nred_batched(const InstDesc* __restrict__ D,
                                                   const Item* __restrict__ it) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  const int idx = w.x * 256 + threadIdx.x;
  if (idx < q.M * q.nb) near_reduce_entry(q.noff, q.npart, q.nb, q.pN, idx);
}

__global__ void __launch_bounds__(256) cxr_batched(const InstDesc* __restrict__ D,
                                                   const Item* __restrict__ it) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  cx_reduce_block(q.g, q.pC, q.c_nchunks, q.gvec, w.x);
}

// rows [4 x, 4 x + 4) of W (rows x cols, row-major) times v: one wavefront per row.
__device__ inline void gemv_rows_block(const cd* __restrict__ W, const cd* __restrict__ v, cd* y,
                                       int rows, int cols, int bx) {
  int row = bx * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const cd* w = W + (size_t)row * cols;
  // four independent partial sums: four row segments in flight per lane
  double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
  int k = lane;
  for (; k + 192 < cols; k += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const cd a = w[k + 64 * u], b = v[k + 64 * u];
      ar[u] = fma(a.r, b.r, ar[u]);
      ar[u] = fma(-a.i, b.i, ar[u]);
      ai[u] = fma(a.r, b.i, ai[u]);
      ai[u] = fma(a.i, b.r, ai[u]);
    }
  }
  for (; k < cols; k += 64) {
    const cd a = w[k], b = v[k];
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
  if (lane == 0) y[row] = cd{sr, si};
}

// t = Sigma^+ U^* g (g = f for the right-hand side), then w = E V t
__global__ void __launch_bounds__(256) gemv1_batched(const InstDesc* __restrict__ D,
                                                     const Item* __restrict__ it, int use_f) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  gemv_rows_block(q.W1, use_f ? q.f : q.gvec, q.tvec, q.rank, q.n_g, w.x);
}
__global__ void __launch_bounds__(256) gemv2_batched(const InstDesc* __restrict__ D,
                                                     const Item* __restrict__ it) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  gemv_rows_block(q.W2, q.tvec, q.wvec, q.n_b, q.rank, w.x);
}

template <int P>
__global__ void __launch_bounds__(64 * BX_WAVES) bx_batched(const InstDesc* __restrict__ D,
                                                 const Item* __restrict__ it) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  bx_block<P>(q.g, q.cx, q.cy, q.wvec, q.pB, q.b_chunk, q.htab, w.x, w.y);
}

__global__ void __launch_bounds__(256) l2l_batched(const InstDesc* __restrict__ D,
                                                  const Item* __restrict__ it) {
  const Item w = it[blockIdx.x];
  const InstDesc& q = D[w.inst];
  if (!q.active) return;
  l2l_block(q.M, q.P, q.Q2, q.l2l, q.wvec + q.g.col_off[CB_A2], q.pL, w.x, w.y);
}

// sum_{c < n} part[c stride + i] as four interleaved partial sums (c mod 4), so that
// four loads are in flight; fixed order
template <typename TT>
__device__ __forceinline__ cd chunks_sum(const TT* __restrict__ part, int n, size_t stride,
                                         int64_t i) {
  cd s[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  int c = 0;
  for (; c + 3 < n; c += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const TT v = part[(size_t)(c + u) * stride + i];
      s[u].r += v.r;
      s[u].i += v.i;
    }
  }
  for (; c < n; ++c) {
    const TT v = part[(size_t)c * stride + i];
    s[0].r += v.r;
    s[0].i += v.i;
  }
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// Y = D o (x - s o (T x - B x)) with x = X (already un-normalised) for mode 0, or
// Y = D o (s o B f) for the right-hand side (mode 1).  Padding entries get 0.
__global__ void __launch_bounds__(BT) combine_batched(const InstDesc* __restrict__ D,
                                                      const int* __restrict__ seg2inst,
                                                      const cd* __restrict__ X,
                                                      const double* __restrict__ dn, cd* Y,
                                                      int mode) {
  const int seg = blockIdx.x;
  const InstDesc& q = D[seg2inst[seg]];
  for (int r = 0; r < SEG / BT; ++r) {
    const int64_t i = (int64_t)seg * SEG + r * BT + threadIdx.x;
    const int64_t loc = i - q.off;
    if (loc >= q.nbeta || (mode == 0 && !q.active)) {
      Y[i] = cd{0.0, 0.0};
      continue;
    }
    const cd b = q.pL[loc] + chunks_sum(q.pB, q.b_nchunks, q.nbeta, loc);
    cd y;
    if (mode == 0) {
      const cd t = chunks_sum(q.pT, q.m2l_nchunks, q.nbeta, loc);
      if (q.sblk) {   // dense blocks: w here, y in sblock_batched
        q.wS[loc] = t - b;
        continue;
      }
      y = X[i] - q.mie[loc] * (t - b);
    } else {
      if (q.sblk) {
        q.wS[loc] = b;
        continue;
      }
      y = q.mie[loc] * b;
    }
    Y[i] = dn[i] * y;
  }
}

// Second pass for the problems with dense scattering-matrix blocks:
// Y = D o (x - S w) (mode 0) or Y = D o (S w) (mode 1), w from the combine.
__global__ void __launch_bounds__(BT) sblock_batched(const InstDesc* __restrict__ D,
                                                     const int* __restrict__ seg2inst,
                                                     const cd* __restrict__ X,
                                                     const double* __restrict__ dn, cd* Y,
                                                     int mode) {
  const int seg = blockIdx.x;
  const InstDesc& q = D[seg2inst[seg]];
  if (!q.sblk || (mode == 0 && !q.active)) return;
  const int nb = q.nb;
  for (int r = 0; r < SEG / BT; ++r) {
    const int64_t i = (int64_t)seg * SEG + r * BT + threadIdx.x;
    const int64_t loc = i - q.off;
    if (loc >= q.nbeta) continue;
    const int64_t j = loc / nb;
    const cd* row = q.sblk + (size_t)loc * nb;
    const cd* wj = q.wS + (size_t)j * nb;
    cd acc{0.0, 0.0};
    for (int n = 0; n < nb; ++n) cmac(acc, row[n], wj[n]);
    Y[i] = dn[i] * (mode == 0 ? X[i] - acc : acc);
  }
}

// The mixed-precision apply, Y = D o (x - s o ((T32 x + T_near x) - B x)): FP32
// partials of the well-separated pairs plus the FP64 near-pair sums.
__global__ void __launch_bounds__(BT) combine_mixed_batched(const InstDesc* __restrict__ D,
                                                            const int* __restrict__ seg2inst,
                                                            const cd* __restrict__ X,
                                                            const double* __restrict__ dn, cd* Y) {
  const int seg = blockIdx.x;
  const InstDesc& q = D[seg2inst[seg]];
  for (int r = 0; r < SEG / BT; ++r) {
    const int64_t i = (int64_t)seg * SEG + r * BT + threadIdx.x;
    const int64_t loc = i - q.off;
    if (loc >= q.nbeta || !q.active) {
      Y[i] = cd{0.0, 0.0};
      continue;
    }
    const cd b = q.pL[loc] + chunks_sum(q.pB, q.b_nchunks, q.nbeta, loc);
    const cd t = q.pN[loc] + chunks_sum(q.pT32, q.m2l_nchunks, q.nbeta, loc);
    if (q.sblk) {   // dense blocks: w here, y in sblock_batched
      q.wS[loc] = t - b;
      continue;
    }
    Y[i] = dn[i] * (X[i] - q.mie[loc] * (t - b));
  }
}

// ---------------------------------------------------------------------------
// batched Krylov kernels (concatenated vectors, per-problem reductions)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(BT) ew_to32_kernel(const cd* x, cf* y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i < n) y[i] = cf{(float)x[i].r, (float)x[i].i};
}
__global__ void __launch_bounds__(BT) ew_add_kernel(cd* x, const cd* e, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i < n) x[i] += e[i];
}

__global__ void __launch_bounds__(BT) ew_scale_kernel(const cd* x, const double* d, cd* y,
                                                      int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i < n) y[i] = d[i] * x[i];
}
__global__ void __launch_bounds__(BT) ew_sub_kernel(const cd* a, const cd* b, cd* o, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
  if (i < n) o[i] = a[i] - b[i];
}

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int t = 0; t < BT / 64; ++t) s += red[t];
  return s;
}

// The Krylov kernels below skip the segments of inactive problems (their results are
// no longer used) and report zero for them.

// partial[seg] = sum over the segment of |x|^2
__global__ void __launch_bounds__(BT) seg_norm2_kernel(const InstDesc* __restrict__ D,
                                                       const int* __restrict__ seg2inst,
                                                       const cd* __restrict__ x, double* partial) {
  __shared__ double red[BT / 64];
  if (!D[seg2inst[blockIdx.x]].active) {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  double s = 0.0;
  for (int r = 0; r < SEG / BT; ++r) s += cabs2(x[(int64_t)blockIdx.x * SEG + r * BT + threadIdx.x]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// nrm[i] = sqrt(sum of the segments of problem i)
__global__ void inst_norm_kernel(const InstDesc* __restrict__ D, int B, const double* partial,
                                 double* nrm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  double s = 0.0;
  for (int g = D[i].seg0; g < D[i].seg0 + D[i].nseg; ++g) s += partial[g];
  nrm[i] = sqrt(s);
}

// y = x / nrm[problem] (where nrm > 0)
__global__ void __launch_bounds__(BT) inst_scale_kernel(const InstDesc* __restrict__ D,
                                                        const int* __restrict__ seg2inst,
                                                        const cd* x, const double* nrm, cd* y) {
  if (!D[seg2inst[blockIdx.x]].active) return;
  const double s = nrm[seg2inst[blockIdx.x]];
  for (int r = 0; r < SEG / BT; ++r) {
    int64_t i = (int64_t)blockIdx.x * SEG + r * BT + threadIdx.x;
    y[i] = s > 0 ? (1.0 / s) * x[i] : x[i];
  }
}

// partial[v][seg] = sum over the segment of conj(V_v) w, v = 0..nv-1; block (seg, y)
// takes v in [y DOT_VB, y DOT_VB + DOT_VB)
constexpr int DOT_VB = 8;
__global__ void __launch_bounds__(BT) seg_dots_kernel(const InstDesc* __restrict__ D,
                                                      const int* __restrict__ seg2inst,
                                                      const cd* __restrict__ V, size_t ldv,
                                                      const cd* __restrict__ w, int nv, int nseg,
                                                      cd* partial) {
  __shared__ double red[BT / 64];
  const int v0 = blockIdx.y * DOT_VB, v1 = min(nv, v0 + DOT_VB);
  if (!D[seg2inst[blockIdx.x]].active) {
    for (int v = v0 + threadIdx.x; v < v1; v += BT) partial[(size_t)v * nseg + blockIdx.x] = cd{0, 0};
    return;
  }
  cd wv[SEG / BT];
  for (int r = 0; r < SEG / BT; ++r) wv[r] = w[(int64_t)blockIdx.x * SEG + r * BT + threadIdx.x];
  for (int v = v0; v < v1; ++v) {
    const cd* a = V + (size_t)v * ldv + (int64_t)blockIdx.x * SEG;
    double sr = 0.0, si = 0.0;
    for (int r = 0; r < SEG / BT; ++r) {
      cd x = a[r * BT + threadIdx.x];
      sr = fma(x.r, wv[r].r, sr);
      sr = fma(x.i, wv[r].i, sr);
      si = fma(x.r, wv[r].i, si);
      si = fma(-x.i, wv[r].r, si);
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    if (threadIdx.x == 0) partial[(size_t)v * nseg + blockIdx.x] = cd{sr, si};
  }
}

// h[i][v] = sum over problem i's segments of partial[v][.]; H column j += h (pass 1)
__global__ void inst_dots_kernel(const InstDesc* __restrict__ D, int B, int nv, int nseg,
                                 const cd* partial, cd* h, int hld, cd* H, int ldh, int j,
                                 int pass) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * nv) return;
  int i = idx / nv, v = idx - i * nv;
  cd s{0, 0};
  for (int g = D[i].seg0; g < D[i].seg0 + D[i].nseg; ++g) s += partial[(size_t)v * nseg + g];
  h[(size_t)i * hld + v] = s;
  cd* hc = H + (size_t)i * ldh * ldh + (size_t)j * ldh;
  hc[v] = pass ? hc[v] + s : s;
}

// w -= sum_v h[problem][v] V_v
__global__ void __launch_bounds__(BT) seg_update_kernel(const InstDesc* __restrict__ D,
                                                        const int* __restrict__ seg2inst,
                                                        const cd* __restrict__ V, size_t ldv,
                                                        cd* w, int nv, const cd* __restrict__ h,
                                                        int hld) {
  // block (seg, r): entries [seg SEG + r BT, seg SEG + (r+1) BT), one per thread
  if (!D[seg2inst[blockIdx.x]].active) return;
  const cd* hh = h + (size_t)seg2inst[blockIdx.x] * hld;
  const int64_t i = (int64_t)blockIdx.x * SEG + blockIdx.y * BT + threadIdx.x;
  cd acc = w[i];
  for (int v = 0; v < nv; ++v) {
    cd hv = hh[v];
    cd a = V[(size_t)v * ldv + i];
    acc.r -= hv.r * a.r - hv.i * a.i;
    acc.i -= hv.r * a.i + hv.i * a.r;
  }
  w[i] = acc;
}

// Per problem: rotations of column j of its Hessenberg matrix (as in the single
// solver) and res[i][j] = |g[j+1]|; hn[i] = H[j+1][j].
__global__ void inst_givens_kernel(int B, const double* nrm, cd* H, int ldh, cd* cs, cd* sn, cd* g,
                                   int j, double* hn, double* res, int rld) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  cd* Hi = H + (size_t)i * ldh * ldh;
  cd* csi = cs + (size_t)i * ldh;
  cd* sni = sn + (size_t)i * ldh;
  cd* gi = g + (size_t)i * (ldh + 1);
  double hnorm = nrm[i];
  hn[i] = hnorm;
  cd* h = Hi + (size_t)j * ldh;
  h[j + 1] = cd{hnorm, 0.0};
  for (int t = 0; t < j; ++t) {
    cd u = conj(csi[t]) * h[t] + conj(sni[t]) * h[t + 1];
    h[t + 1] = -(sni[t] * h[t]) + csi[t] * h[t + 1];
    h[t] = u;
  }
  cd a = h[j], b = h[j + 1];
  double den = sqrt(cabs2(a) + cabs2(b));
  cd c = den > 0 ? (1.0 / den) * a : cd{1.0, 0.0};
  cd s = den > 0 ? (1.0 / den) * b : cd{0.0, 0.0};
  csi[j] = c;
  sni[j] = s;
  h[j] = cd{den, 0.0};
  h[j + 1] = cd{0.0, 0.0};
  gi[j + 1] = -(s * gi[j]);
  gi[j] = conj(c) * gi[j];
  res[(size_t)i * rld + j] = sqrt(cabs2(gi[j + 1]));
}

__global__ void inst_init_g_kernel(int B, int len, const double* beta, cd* g) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * len) return;
  int i = idx / len, t = idx - i * len;
  g[idx] = (t == 0) ? cd{beta[i], 0.0} : cd{0.0, 0.0};
}

__global__ void inst_backsolve_kernel(int B, const cd* H, int ldh, const cd* g, const int* kk,
                                      cd* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const cd* Hi = H + (size_t)i * ldh * ldh;
  const cd* gi = g + (size_t)i * (ldh + 1);
  cd* yi = y + (size_t)i * ldh;
  int k = kk[i];
  for (int r = k - 1; r >= 0; --r) {
    cd s = gi[r];
    for (int t = r + 1; t < k; ++t) s -= Hi[(size_t)t * ldh + r] * yi[t];
    cd dd = Hi[(size_t)r * ldh + r];
    yi[r] = (cabs2(dd) > 0) ? cdiv(s, dd) : cd{0.0, 0.0};
  }
}

// x += sum_{v < k[problem]} y[problem][v] V_v
__global__ void __launch_bounds__(BT) seg_axpy_basis_kernel(const int* __restrict__ seg2inst,
                                                            cd* x, const cd* __restrict__ V,
                                                            size_t ldv, const cd* __restrict__ y,
                                                            int yld, const int* __restrict__ kk) {
  // block (seg, r): entries [seg SEG + r BT, seg SEG + (r+1) BT), one per thread
  const int i0 = seg2inst[blockIdx.x];
  const int k = kk[i0];
  const cd* yy = y + (size_t)i0 * yld;
  const int64_t i = (int64_t)blockIdx.x * SEG + blockIdx.y * BT + threadIdx.x;
  cd acc = x[i];
  for (int v = 0; v < k; ++v) cmac(acc, yy[v], V[(size_t)v * ldv + i]);
  x[i] = acc;
}

// D[i].active = flags[i]
__global__ void set_active_kernel(InstDesc* D, const int* __restrict__ flags, int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) D[i].active = flags[i];
}

// x = 0 on the segments of problems whose flag is set
__global__ void __launch_bounds__(BT) zero_rejected_kernel(const int* __restrict__ seg2inst,
                                                           const int* __restrict__ flag, cd* x) {
  if (!flag[seg2inst[blockIdx.x]]) return;
  for (int r = 0; r < SEG / BT; ++r) x[(int64_t)blockIdx.x * SEG + r * BT + threadIdx.x] = cd{0.0, 0.0};
}


}  // namespace

struct grt_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<grt_ctx*> ctx;
  int B = 0;
  std::vector<InstDesc> hd;
  InstDesc* dd = nullptr;
  int64_t ntot = 0;
  int nseg = 0;
  int* d_seg2inst = nullptr;
  double *d_dnorm = nullptr, *d_dinv = nullptr;
  struct Group {
    int P;
    // m2l / m2lt32: translation items of the problems without / with an FP32 table
    // (the mixed apply's FP32 launches); m2lf / m2lh / m2lt: those of the problems on
    // the fly in one launch / on the fly split over two half-output launches / with a
    // resident table (FP64 apply)
    Item *m2l = nullptr, *m2lt32 = nullptr, *m2lf = nullptr, *m2lh = nullptr, *m2lt = nullptr,
         *cx = nullptr, *bx = nullptr, *nr = nullptr;
    int n_m2l = 0, n_m2lt32 = 0, n_m2lf = 0, n_m2lh = 0, n_m2lt = 0, n_cx = 0, n_bx = 0,
        n_nr = 0;
  };
  std::vector<uint64_t> gen;  // the contexts' generations at creation
  std::vector<Group> groups;
  Item *it_cxr = nullptr, *it_g1 = nullptr, *it_g2 = nullptr, *it_l2l = nullptr, *it_nred = nullptr;
  int n_cxr = 0, n_g1 = 0, n_g2 = 0, n_l2l = 0, n_nred = 0;
  cf* x32 = nullptr;      // FP32 copy of the apply's input (mixed precision)
  size_t l2l_smem = 0;
  // Krylov workspace
  int m = 0;
  cd* V = nullptr;        // m + 7 slots of ntot: basis 0..m, iterate, rhs, apply in, out,
                          // refinement residual and correction
  cd *xtmp = nullptr, *wout = nullptr;   // slots m+3, m+4: the apply's fixed buffers
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // captured batch_apply_core: FP64, mixed
  cd* H = nullptr;        // B x (m+1)^2
  cd *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *h = nullptr;
  double *res = nullptr, *part = nullptr, *nrm = nullptr, *hn = nullptr, *bn = nullptr;
  cd* dpart = nullptr;    // (m+1) x nseg
  int* d_k = nullptr;
  int* d_act = nullptr;         // staging of the active flags
  std::vector<int> act;         // the flags as last sent to the descriptors
  double* h_pinned = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // angles of one geometry (a context with several right-hand sides): the mixed
  // apply translates all of them at once on the owner's FP32 matrix-core product
  grt_ctx* block_owner = nullptr;
  int64_t block_stride = 0;   // distance between consecutive instances' vectors
  bool any_shapes = false;    // some problem has dense scattering-matrix blocks
};

static grt_status bset(grt_batch* b, grt_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}
#define BHIP(b, call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return bset(b, GRT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)
#define BTRY(x)                  \
  do {                           \
    grt_status s_ = (x);         \
    if (s_ != GRT_OK) return s_; \
  } while (0)

template <typename T>
static grt_status upload(grt_batch* b, const std::vector<T>& v, T** out) {
  BHIP(b, hipMalloc(out, sizeof(T) * std::max<size_t>(1, v.size())));
  if (!v.empty()) BHIP(b, hipMemcpy(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return GRT_OK;
}

#define BATCH_P_DISPATCH(FN, P, ...)                          \
  switch (P) {                                                \
    case 1: FN<1>(__VA_ARGS__); break;                        \
    case 2: FN<2>(__VA_ARGS__); break;                        \
    case 3: FN<3>(__VA_ARGS__); break;                        \
    case 4: FN<4>(__VA_ARGS__); break;                        \
    case 5: FN<5>(__VA_ARGS__); break;                        \
    case 6: FN<6>(__VA_ARGS__); break;                        \
    case 8: FN<8>(__VA_ARGS__); break;                        \
    case 10: FN<10>(__VA_ARGS__); break;                      \
    case 12: FN<12>(__VA_ARGS__); break;                      \
    case 15: FN<15>(__VA_ARGS__); break;                      \
    case 20: FN<20>(__VA_ARGS__); break;                      \
    default: return bset(b, GRT_EUNSUP, "P not compiled in"); \
  }

template <int P>
static void launch_group_T(grt_batch* b, const grt_batch::Group& gp, const cd* X) {
  if (gp.n_m2lf) m2l_batched<P><<<gp.n_m2lf, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2lf, X);
  if (gp.n_m2lh) {
    constexpr int NB = 2 * P + 1, H0 = (NB + 1) / 2;
    m2lh_batched<P, 0, H0><<<gp.n_m2lh, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2lh, X);
    m2lh_batched<P, H0, NB - H0><<<gp.n_m2lh, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2lh, X);
  }
  if (gp.n_m2lt) m2lt_batched<P><<<gp.n_m2lt, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2lt, X);
}
template <int P>
static void launch_group_C(grt_batch* b, const grt_batch::Group& gp, const cd* X) {
  if (gp.n_cx) cx_batched<P><<<gp.n_cx, 64 * CX_WAVES, 0, b->stream>>>(b->dd, gp.cx, X);
}
template <int P>
static void launch_group_B(grt_batch* b, const grt_batch::Group& gp) {
  if (gp.n_bx) bx_batched<P><<<gp.n_bx, 64 * BX_WAVES, 0, b->stream>>>(b->dd, gp.bx);
}
template <int P>
static void launch_group_T32(grt_batch* b, const grt_batch::Group& gp) {
  if (gp.n_m2l) m2l32_batched<P><<<gp.n_m2l, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2l, b->x32);
  if (gp.n_m2lt32)
    m2lt32_batched<P><<<gp.n_m2lt32, M2L_THREADS, 0, b->stream>>>(b->dd, gp.m2lt32, b->x32);
  if (gp.n_nr) near_batched<P><<<gp.n_nr, 64, 0, b->stream>>>(b->dd, gp.nr, b->xtmp);
}

// layer correction tail for all problems: t = W1 g (or f), w = W2 t, then B and L2L
static grt_status batch_lowrank(grt_batch* b, int use_f) {
  hipStream_t s = b->stream;
  if (b->n_g1) gemv1_batched<<<b->n_g1, 256, 0, s>>>(b->dd, b->it_g1, use_f);
  if (b->n_g2) gemv2_batched<<<b->n_g2, 256, 0, s>>>(b->dd, b->it_g2);
  for (auto& gp : b->groups) BATCH_P_DISPATCH(launch_group_B, gp.P, b, gp);
  if (b->n_l2l) l2l_batched<<<b->n_l2l, 256, b->l2l_smem, s>>>(b->dd, b->it_l2l);
  BHIP(b, hipGetLastError());
  return GRT_OK;
}

// The mixed apply of a block of angles, Y = D x - Yb + D s B x, with Yb = D S T D^{-1}
// (D x) from the matrix-core product (column r = instance r).
__global__ void __launch_bounds__(BT) combine_block_batched(const InstDesc* __restrict__ D,
                                                            const int* __restrict__ seg2inst,
                                                            const cd* __restrict__ X,
                                                            const double* __restrict__ dn,
                                                            const cf* __restrict__ Yb, int Rp,
                                                            cd* Y) {
  const int seg = blockIdx.x;
  const int inst = seg2inst[seg];
  const InstDesc& q = D[inst];
  for (int r = 0; r < SEG / BT; ++r) {
    const int64_t i = (int64_t)seg * SEG + r * BT + threadIdx.x;
    const int64_t loc = i - q.off;
    if (loc >= q.nbeta || !q.active) {
      Y[i] = cd{0.0, 0.0};
      continue;
    }
    const cd b = q.pL[loc] + chunks_sum(q.pB, q.b_nchunks, q.nbeta, loc);
    const cf t = Yb[(size_t)loc * Rp + inst];
    Y[i] = dn[i] * (X[i] + q.mie[loc] * b) - cd{t.r, t.i};
  }
}

// wout = D K D^{-1} x for every problem, x = D^{-1} xh already in xtmp (both fixed
// buffers of the batch, so the whole launch sequence can be captured once as a HIP
// graph and replayed; see batch_apply).
// With mixed: the translation of well-separated pairs in FP32 (FP32 copy of x, FP32
// accumulation) and of near pairs in FP64; C x, A^+ and B_phys w in FP64 as always.
static grt_status batch_apply_core(grt_batch* b, bool mixed) {
  hipStream_t s = b->stream;
  if (mixed && b->block_owner) {
    grt_ctx* o = b->block_owner;
    grt_status st = block_product(o, b->xtmp, b->block_stride, o->d_dnorm, b->B, s);
    if (st != GRT_OK) return bset(b, st, "block translation: " + o->err);
    for (auto& gp : b->groups) BATCH_P_DISPATCH(launch_group_C, gp.P, b, gp, b->xtmp);
    if (b->n_cxr) cxr_batched<<<b->n_cxr, 256, 0, s>>>(b->dd, b->it_cxr);
    BTRY(batch_lowrank(b, 0));
    combine_block_batched<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, b->xtmp, b->d_dnorm,
                                                 o->d_blkY, o->blk_Rp, b->wout);
    BHIP(b, hipGetLastError());
    return GRT_OK;
  }
  if (mixed) {
    const unsigned gn = (unsigned)((b->ntot + BT - 1) / BT);
    ew_to32_kernel<<<gn, BT, 0, s>>>(b->xtmp, b->x32, b->ntot);
    for (auto& gp : b->groups) BATCH_P_DISPATCH(launch_group_T32, gp.P, b, gp);
    if (b->n_nred) nred_batched<<<b->n_nred, 256, 0, s>>>(b->dd, b->it_nred);
  } else {
    for (auto& gp : b->groups) BATCH_P_DISPATCH(launch_group_T, gp.P, b, gp, b->xtmp);
  }
  for (auto& gp : b->groups) BATCH_P_DISPATCH(launch_group_C, gp.P, b, gp, b->xtmp);
  if (b->n_cxr) cxr_batched<<<b->n_cxr, 256, 0, s>>>(b->dd, b->it_cxr);
  BTRY(batch_lowrank(b, 0));
  if (mixed)
    combine_mixed_batched<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, b->xtmp, b->d_dnorm,
                                                 b->wout);
  else
    combine_batched<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, b->xtmp, b->d_dnorm, b->wout, 0);
  if (b->any_shapes)
    sblock_batched<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, b->xtmp, b->d_dnorm, b->wout, 0);
  BHIP(b, hipGetLastError());
  return GRT_OK;
}

// wout = D K D^{-1} xh (xh concatenated; K the mixed-precision operator if mixed),
// the core replayed from a graph if asked
static grt_status batch_apply(grt_batch* b, const cd* xh, bool use_graph, bool mixed) {
  hipStream_t s = b->stream;
  const unsigned gn = (unsigned)((b->ntot + BT - 1) / BT);
  ew_scale_kernel<<<gn, BT, 0, s>>>(xh, b->d_dinv, b->xtmp, b->ntot);
  if (!use_graph) return batch_apply_core(b, mixed);
  hipGraphExec_t& ge = b->graph[mixed ? 1 : 0];
  if (!ge) {
    hipGraph_t gr = nullptr;
    BHIP(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    grt_status st = batch_apply_core(b, mixed);
    hipError_t e = hipStreamEndCapture(s, &gr);
    if (st != GRT_OK || e != hipSuccess) {
      if (gr) hipGraphDestroy(gr);
      return st != GRT_OK ? st : bset(b, GRT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (e != hipSuccess) {
      ge = nullptr;
      return bset(b, GRT_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
  }
  BHIP(b, hipGraphLaunch(ge, s));
  return GRT_OK;
}

static grt_status batch_rhs_hat(grt_batch* b, cd* Y) {
  BTRY(batch_lowrank(b, 1));
  combine_batched<<<b->nseg, BT, 0, b->stream>>>(b->dd, b->d_seg2inst, nullptr, b->d_dnorm, Y, 1);
  if (b->any_shapes)
    sblock_batched<<<b->nseg, BT, 0, b->stream>>>(b->dd, b->d_seg2inst, nullptr, b->d_dnorm, Y, 1);
  BHIP(b, hipGetLastError());
  return GRT_OK;
}

static grt_status batch_norms(grt_batch* b, const cd* x, double* nrm_dev) {
  seg_norm2_kernel<<<b->nseg, BT, 0, b->stream>>>(b->dd, b->d_seg2inst, x, b->part);
  inst_norm_kernel<<<(b->B + 63) / 64, 64, 0, b->stream>>>(b->dd, b->B, b->part, nrm_dev);
  BHIP(b, hipGetLastError());
  return GRT_OK;
}

static grt_status batch_workspace(grt_batch* b, int m) {
  if (b->m == m && b->V) return GRT_OK;
  void* olds[] = {b->V, b->H, b->cs, b->sn, b->g, b->y, b->h, b->res, b->part, b->nrm, b->hn,
                  b->bn, b->dpart, b->d_k};
  for (void* p : olds)
    if (p) hipFree(p);
  const size_t B = b->B, n = b->ntot, ld = m + 1;
  for (hipGraphExec_t& ge : b->graph)  // the captured applies point into the old workspace
    if (ge) {
      hipGraphExecDestroy(ge);
      ge = nullptr;
    }
  BHIP(b, hipMalloc(&b->V, sizeof(cd) * n * (m + 7)));
  b->xtmp = b->V + n * (m + 3);
  b->wout = b->V + n * (m + 4);
  BHIP(b, hipMalloc(&b->H, sizeof(cd) * B * ld * ld));
  BHIP(b, hipMalloc(&b->cs, sizeof(cd) * B * ld));
  BHIP(b, hipMalloc(&b->sn, sizeof(cd) * B * ld));
  BHIP(b, hipMalloc(&b->g, sizeof(cd) * B * (ld + 1)));
  BHIP(b, hipMalloc(&b->y, sizeof(cd) * B * ld));
  BHIP(b, hipMalloc(&b->h, sizeof(cd) * B * ld));
  BHIP(b, hipMalloc(&b->res, sizeof(double) * B * ld));
  BHIP(b, hipMalloc(&b->part, sizeof(double) * b->nseg));
  BHIP(b, hipMalloc(&b->nrm, sizeof(double) * B));
  BHIP(b, hipMalloc(&b->hn, sizeof(double) * B));
  BHIP(b, hipMalloc(&b->bn, sizeof(double) * B));
  BHIP(b, hipMalloc(&b->dpart, sizeof(cd) * ld * b->nseg));
  BHIP(b, hipMalloc(&b->d_k, sizeof(int) * B));
  if (!b->h_pinned) BHIP(b, hipHostMalloc(&b->h_pinned, sizeof(double) * 3 * B + 64));
  if (!b->ev[0]) {
    BHIP(b, hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming));
    BHIP(b, hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming));
  }
  b->m = m;
  return GRT_OK;
}

// Send the problems' active flags to the descriptors (only if they changed).
static grt_status set_active(grt_batch* b, const std::vector<int>& flags) {
  if (flags == b->act) return GRT_OK;
  BHIP(b, hipMemcpyAsync(b->d_act, flags.data(), sizeof(int) * b->B, hipMemcpyHostToDevice,
                         b->stream));
  set_active_kernel<<<(b->B + 63) / 64, 64, 0, b->stream>>>(b->dd, b->d_act, b->B);
  BHIP(b, hipGetLastError());
  b->act = flags;
  return GRT_OK;
}

static grt_status read_vec(grt_batch* b, const double* dev, std::vector<double>& out) {
  out.resize(b->B);
  BHIP(b, hipMemcpyAsync(b->h_pinned, dev, sizeof(double) * b->B, hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  std::memcpy(out.data(), b->h_pinned, sizeof(double) * b->B);
  return GRT_OK;
}

// Per-problem outcome of a lockstep GMRES run.
struct LockstepResult {
  std::vector<int> iters, cycles, rejected;
  std::vector<double> rel;
  int steps = 0;  // lockstep Arnoldi steps taken (the longest problem's count)
  explicit LockstepResult(int B) : iters(B, 0), cycles(B, 0), rejected(B, 0), rel(B, 1.0) {}
};

// Restarted GMRES for all problems in lockstep on D K D^{-1} X = Bv (K the mixed
// operator if mixed): X (normalised, in place) from its current value.  A problem
// stops updating once its residual estimate reaches tol ||Bv_i|| (a problem with
// Bv_i = 0 is done at once).  With guard, an initial X_i no better than zero is
// dropped and that problem restarts from zero.  With relax > 0 (relaxed inexact
// GMRES, FP64 operator): an Arnoldi step applies the mixed operator once every
// problem still iterating has a residual estimate at most relax ||Bv_i||; the
// residuals at the restarts stay FP64.
static grt_status batch_gmres(grt_batch* b, bool mixed, const cd* Bv, cd* X, double tol,
                              int maxit, int m, bool guard, bool use_graph, LockstepResult& r,
                              double relax = 0.0, int* fast_steps = nullptr) {
  hipStream_t s = b->stream;
  const int B = b->B, ld = m + 1;
  const size_t ldv = (size_t)b->ntot;
  cd* V = b->V;
  BTRY(batch_norms(b, Bv, b->bn));
  std::vector<double> bn, beta0;
  BTRY(read_vec(b, b->bn, bn));
  std::vector<int> kk(B, 0);
  std::vector<char> done(B, 0);
  const std::vector<int> all_on(B, 1);
  std::vector<int> act(B, 1);
  int total = 0;
  while (true) {
    // R = B - K X into V_0 (for every problem)
    BTRY(set_active(b, all_on));
    BTRY(batch_apply(b, X, use_graph, mixed));
    {
      const unsigned gn = (unsigned)((b->ntot + BT - 1) / BT);
      ew_sub_kernel<<<gn, BT, 0, s>>>(Bv, b->wout, V, b->ntot);
    }
    BTRY(batch_norms(b, V, b->nrm));
    BTRY(read_vec(b, b->nrm, beta0));
    bool any = false, reject = false;
    for (int i = 0; i < B; ++i) {
      r.rel[i] = bn[i] > 0 ? beta0[i] / bn[i] : 0.0;
      done[i] = r.rel[i] <= tol;
      if (!done[i]) any = true;
      if (guard && r.rel[i] >= 1.0) {
        r.rejected[i] = 1;
        reject = true;
      }
    }
    if (guard) {
      guard = false;
      if (reject) {
        // initial guesses no better than zero are dropped: those problems restart
        // from x = 0 (the residual is then recomputed for the whole batch)
        BHIP(b, hipMemcpyAsync(b->d_k, r.rejected.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
        zero_rejected_kernel<<<b->nseg, BT, 0, s>>>(b->d_seg2inst, b->d_k, X);
        BHIP(b, hipGetLastError());
        continue;
      }
    }
    if (!any || total >= maxit) break;
    inst_scale_kernel<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, V, b->nrm, V);
    inst_init_g_kernel<<<(B * (ld + 1) + 255) / 256, 256, 0, s>>>(B, ld + 1, b->nrm, b->g);
    BHIP(b, hipMemsetAsync(b->H, 0, sizeof(cd) * (size_t)B * ld * ld, s));
    std::fill(kk.begin(), kk.end(), -1);
    for (int i = 0; i < B; ++i) {
      if (done[i]) kk[i] = 0;
      act[i] = !done[i];
    }
    // problems already at tol take no Arnoldi steps: their applies are skipped
    BTRY(set_active(b, act));
    int steps = 0;
    // residual estimates of step jj, in the pinned buffer of parity jj & 1
    double* hbuf[2] = {b->h_pinned + B, b->h_pinned + 2 * B};
    auto check = [&](int jj) {
      bool all = true;
      for (int i = 0; i < B; ++i) {
        if (kk[i] >= 0) continue;
        if (hbuf[jj & 1][i] <= tol * bn[i]) kk[i] = jj + 1;
        else all = false;
      }
      return all;
    };
    bool all = false;
    // the largest relative residual estimate among the problems still iterating
    double est = 0.0;
    for (int i = 0; i < B; ++i)
      if (!done[i]) est = std::max(est, r.rel[i]);
    for (int j = 0; j < m && total + j < maxit; ++j) {
      cd* w = b->wout;  // the new directions; normalised into V_{j+1} below
      const bool fast = mixed || (relax > 0 && est <= relax);
      if (fast && !mixed && fast_steps) ++*fast_steps;
      BTRY(batch_apply(b, V + (size_t)j * ldv, use_graph, fast));
      for (int pass = 0; pass < 2; ++pass) {
        seg_dots_kernel<<<dim3(b->nseg, (j + 1 + DOT_VB - 1) / DOT_VB), BT, 0, s>>>(
            b->dd, b->d_seg2inst, V, ldv, w, j + 1, b->nseg, b->dpart);
        inst_dots_kernel<<<(B * (j + 1) + 255) / 256, 256, 0, s>>>(b->dd, B, j + 1, b->nseg,
                                                                  b->dpart, b->h, ld, b->H, ld, j,
                                                                  pass);
        seg_update_kernel<<<dim3(b->nseg, SEG / BT), BT, 0, s>>>(b->dd, b->d_seg2inst, V, ldv, w,
                                                                 j + 1, b->h, ld);
      }
      BTRY(batch_norms(b, w, b->nrm));
      inst_givens_kernel<<<(B + 63) / 64, 64, 0, s>>>(B, b->nrm, b->H, ld, b->cs, b->sn, b->g, j,
                                                      b->hn, b->res, ld);
      inst_scale_kernel<<<b->nseg, BT, 0, s>>>(b->dd, b->d_seg2inst, w, b->hn, V + (size_t)(j + 1) * ldv);
      BHIP(b, hipGetLastError());
      BHIP(b, hipMemcpy2DAsync(hbuf[j & 1], sizeof(double), b->res + j, sizeof(double) * ld,
                               sizeof(double), B, hipMemcpyDeviceToHost, s));
      BHIP(b, hipEventRecord(b->ev[j & 1], s));
      steps = j + 1;
      // the host checks step j-1 while the GPU runs step j; problems found converged
      // are skipped from step j+1 on (their solution uses columns < kk only)
      if (j >= 1) {
        BHIP(b, hipEventSynchronize(b->ev[(j - 1) & 1]));
        if (check(j - 1)) {
          all = true;
          break;
        }
        est = 0.0;
        for (int i = 0; i < B; ++i) {
          act[i] = kk[i] < 0;
          if (act[i] && bn[i] > 0) est = std::max(est, hbuf[(j - 1) & 1][i] / bn[i]);
        }
        BTRY(set_active(b, act));
      }
    }
    if (!all && steps > 0) {
      BHIP(b, hipEventSynchronize(b->ev[(steps - 1) & 1]));
      check(steps - 1);
    }
    for (int i = 0; i < B; ++i)
      if (kk[i] < 0) kk[i] = steps;
    total += steps;
    BHIP(b, hipMemcpyAsync(b->d_k, kk.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
    inst_backsolve_kernel<<<(B + 63) / 64, 64, 0, s>>>(B, b->H, ld, b->g, b->d_k, b->y);
    seg_axpy_basis_kernel<<<dim3(b->nseg, SEG / BT), BT, 0, s>>>(b->d_seg2inst, X, V, ldv, b->y,
                                                                 ld, b->d_k);
    BHIP(b, hipGetLastError());
    for (int i = 0; i < B; ++i) {
      r.iters[i] += kk[i];
      if (kk[i] > 0) r.cycles[i] += 1;
    }
  }
  r.steps = total;
  BTRY(set_active(b, all_on));
  return GRT_OK;
}

static grt_status batch_create_impl(grt_batch** out, int64_t n, grt_ctx* const* ctxs,
                                    void* hip_stream);

grt_status batch_create_internal(grt_batch** out, int64_t n, grt_ctx* const* ctxs,
                                 void* hip_stream) {
  return batch_create_impl(out, n, ctxs, hip_stream);
}

grt_status batch_set_block(grt_batch* b, grt_ctx* owner) {
  if (!b || !owner || (int64_t)b->B != owner->n_rhs) return GRT_EINVAL;
  const int64_t stride = b->B > 1 ? b->hd[1].off - b->hd[0].off : 0;
  for (int i = 0; i < b->B; ++i)
    if (b->hd[i].off != i * stride || b->hd[i].M != b->hd[0].M || b->hd[i].P != b->hd[0].P)
      return bset(b, GRT_EINVAL, "block instances must share the geometry and the layout");
  b->block_owner = owner;
  b->block_stride = stride;
  return GRT_OK;
}

static grt_status batch_create_impl(grt_batch** out, int64_t n, grt_ctx* const* ctxs,
                                    void* hip_stream) {
  if (!out || n <= 0 || !ctxs) return GRT_EINVAL;
  *out = nullptr;
  grt_batch* b = new (std::nothrow) grt_batch();
  if (!b) return GRT_ENOMEM;
  b->B = (int)n;
  b->ctx.assign(ctxs, ctxs + n);
  b->device = ctxs[0] ? ctxs[0]->device : 0;
  for (grt_ctx* c : b->ctx) {
    if (!c || !c->built || c->M == 0 || c->device != b->device) {
      delete b;
      return GRT_ESTATE;
    }
  }
  // every instance writes its context's scratch buffers (partials, coupling
  // vectors) during a lockstep apply, so one context may appear only once
  {
    std::vector<grt_ctx*> sorted(b->ctx);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
      delete b;
      return GRT_EINVAL;
    }
  }
  hipSetDevice(b->device);
  if (hip_stream) {
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return GRT_EHIP;
    }
    b->own_stream = true;
  }
  // descriptors and the concatenated layout
  b->hd.resize(n);
  int seg = 0;
  std::vector<int> seg2inst;
  std::map<int, std::vector<int>> byP;
  size_t smem = 0;
  for (int i = 0; i < n; ++i) {
    grt_ctx* c = b->ctx[i];
    hipStreamSynchronize(c->stream);
    InstDesc& q = b->hd[i];
    q.g = c->g;
    q.cx = c->d_cx;
    q.cy = c->d_cy;
    q.htab = c->d_htab;
    q.mie = c->d_mie;
    q.W1 = c->d_W1;
    q.W2 = c->d_W2;
    q.l2l = c->d_l2l;
    q.f = c->d_f;
    q.M = (int)c->M;
    q.P = c->P;
    q.nb = c->nb;
    q.rank = c->rank;
    q.n_g = c->n_g;
    q.n_b = c->n_b;
    q.Q2 = c->g.Q[1];
    q.m2l_chunk = c->m2l_chunk;
    q.m2l_nchunks = c->m2l_nchunks;
    q.c_chunk = c->c_chunk;
    q.c_nchunks = c->c_nchunks;
    q.b_chunk = c->b_chunk;
    q.b_nchunks = c->b_nchunks;
    q.pT = c->d_pT;
    q.pC = c->d_pC;
    q.pB = c->d_pB;
    q.pL = c->d_pL;
    q.gvec = c->d_gvec;
    q.tvec = c->d_tvec;
    q.wvec = c->d_wvec;
    q.nbeta = c->n_beta;
    q.pT32 = c->d_x32 ? c->d_pT32 : nullptr;
    q.npart = c->d_npart;
    q.pN = c->d_pN;
    q.noff = c->d_noff;
    q.nlist = c->d_nlist;
    q.ntgt = c->d_ntgt;
    q.n_near = (int)c->n_near;
    q.zsafe = c->zsafe;
    q.table = c->d_table;
    q.mpad = c->table_mpad;
    q.table32 = c->d_table32;
    q.mpad32 = c->table32_mpad;
    q.sblk = c->d_sblk;
    q.wS = c->d_wS;
    if (c->d_sblk) b->any_shapes = true;
    q.split = c->d_table ? 1 : c->m2l_split;
    q.active = 1;
    q.seg0 = seg;
    q.nseg = (int)((c->n_beta + SEG - 1) / SEG);
    q.off = (int64_t)seg * SEG;
    for (int t = 0; t < q.nseg; ++t) seg2inst.push_back(i);
    seg += q.nseg;
    byP[q.P].push_back(i);
    smem = std::max(smem, l2l_lds_bytes(q.P, q.Q2, l2l_targets_per_block(q.P, q.Q2)));
  }
  b->nseg = seg;
  b->ntot = (int64_t)seg * SEG;
  b->l2l_smem = smem;
  // work items
  std::vector<Item> cxr, g1, g2, l2l, nred;
  for (auto& kv : byP) {
    grt_batch::Group gp;
    gp.P = kv.first;
    std::vector<Item> m2l, m2lt32, m2lf, m2lh, m2lt, cxv, bxv, nr;
    for (int i : kv.second) {
      const InstDesc& q = b->hd[i];
      const int nt = 2 * q.g.N + q.g.Nw[1];
      for (int x = 0; x < (q.n_near + 63) / 64; ++x) nr.push_back({i, x, 0});
      for (int y = 0; y < q.m2l_nchunks; ++y)
        for (int x = 0; x < (q.M + 63) / 64; ++x) {
          (q.table32 ? m2lt32 : m2l).push_back({i, x, y});
          (q.table ? m2lt : q.split == 2 ? m2lh : m2lf).push_back({i, x, y});
        }
      for (int y = 0; y < q.c_nchunks; ++y)
        for (int x = 0; x < (nt + 63) / 64; ++x) cxv.push_back({i, x, y});
      for (int y = 0; y < q.b_nchunks; ++y)
        for (int x = 0; x < (q.M + 63) / 64; ++x) bxv.push_back({i, x, y});
    }
    grt_status st;
    if ((st = upload(b, m2l, &gp.m2l)) != GRT_OK || (st = upload(b, cxv, &gp.cx)) != GRT_OK ||
        (st = upload(b, bxv, &gp.bx)) != GRT_OK || (st = upload(b, nr, &gp.nr)) != GRT_OK ||
        (st = upload(b, m2lf, &gp.m2lf)) != GRT_OK || (st = upload(b, m2lh, &gp.m2lh)) != GRT_OK ||
        (st = upload(b, m2lt, &gp.m2lt)) != GRT_OK ||
        (st = upload(b, m2lt32, &gp.m2lt32)) != GRT_OK) {
      for (void* q : {(void*)gp.m2l, (void*)gp.m2lt32, (void*)gp.m2lf, (void*)gp.m2lh,
                      (void*)gp.m2lt, (void*)gp.cx, (void*)gp.bx, (void*)gp.nr})
        if (q) hipFree(q);
      grt_batch_destroy(b);
      return st;
    }
    gp.n_nr = (int)nr.size();
    gp.n_m2l = (int)m2l.size();
    gp.n_m2lt32 = (int)m2lt32.size();
    gp.n_m2lf = (int)m2lf.size();
    gp.n_m2lh = (int)m2lh.size();
    gp.n_m2lt = (int)m2lt.size();
    gp.n_cx = (int)cxv.size();
    gp.n_bx = (int)bxv.size();
    b->groups.push_back(gp);
  }
  for (int i = 0; i < n; ++i) {
    const InstDesc& q = b->hd[i];
    const int nt = 2 * q.g.N + q.g.Nw[1];
    for (int x = 0; x < (nt + 3) / 4; ++x) cxr.push_back({i, x, 0});
    for (int x = 0; x < (q.rank + 3) / 4; ++x) g1.push_back({i, x, 0});
    for (int x = 0; x < (q.n_b + 3) / 4; ++x) g2.push_back({i, x, 0});
    for (int x = 0; x < (q.M * q.nb + 255) / 256; ++x) nred.push_back({i, x, 0});
    {
      const int ntb = l2l_targets_per_block(q.P, q.Q2);  // carried in the item's y
      for (int x = 0; x < (q.M + ntb - 1) / ntb; ++x) l2l.push_back({i, x, ntb});
    }
  }
  // concatenated normalisation
  std::vector<double> dn(b->ntot, 0.0), di(b->ntot, 0.0);
  for (int i = 0; i < n; ++i) {
    grt_ctx* c = b->ctx[i];
    const InstDesc& q = b->hd[i];
    hipMemcpy(dn.data() + q.off, c->d_dnorm, sizeof(double) * q.nbeta, hipMemcpyDeviceToHost);
    hipMemcpy(di.data() + q.off, c->d_dinv, sizeof(double) * q.nbeta, hipMemcpyDeviceToHost);
  }
  grt_status st;
  if ((st = upload(b, cxr, &b->it_cxr)) != GRT_OK || (st = upload(b, g1, &b->it_g1)) != GRT_OK ||
      (st = upload(b, g2, &b->it_g2)) != GRT_OK || (st = upload(b, l2l, &b->it_l2l)) != GRT_OK ||
      (st = upload(b, seg2inst, &b->d_seg2inst)) != GRT_OK ||
      (st = upload(b, nred, &b->it_nred)) != GRT_OK ||
      (st = upload(b, b->hd, &b->dd)) != GRT_OK || (st = upload(b, dn, &b->d_dnorm)) != GRT_OK ||
      (st = upload(b, di, &b->d_dinv)) != GRT_OK) {
    grt_batch_destroy(b);
    return st;
  }
  b->n_cxr = (int)cxr.size();
  b->n_g1 = (int)g1.size();
  b->n_g2 = (int)g2.size();
  b->n_l2l = (int)l2l.size();
  b->n_nred = (int)nred.size();
  b->act.assign(n, 1);
  for (grt_ctx* c : b->ctx) b->gen.push_back(c->gen);
  if (hipMalloc(&b->d_act, sizeof(int) * (size_t)n) != hipSuccess ||
      hipMalloc(&b->x32, sizeof(cf) * (size_t)b->ntot) != hipSuccess) {
    grt_batch_destroy(b);
    return GRT_ENOMEM;
  }
  *out = b;
  return GRT_OK;
}

extern "C" {

grt_status grt_batch_create(grt_batch** out, int64_t n, grt_ctx* const* ctxs, void* hip_stream) {
  if (!out || n <= 0 || !ctxs) return GRT_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (ctxs[i] && ctxs[i]->n_rhs > 1) return GRT_EINVAL;   // its solves batch its angles
    if (ctxs[i] && ctxs[i]->fmm_on) return GRT_EUNSUP;      // batches run the dense translation
  }
  return batch_create_impl(out, n, ctxs, hip_stream);
}

grt_status grt_batch_destroy(grt_batch* b) {
  if (!b) return GRT_OK;
  hipSetDevice(b->device);
  if (b->stream) hipStreamSynchronize(b->stream);
  std::vector<void*> p = {b->dd, b->d_seg2inst, b->d_dnorm, b->d_dinv, b->it_cxr, b->it_g1,
                          b->it_g2, b->it_l2l, b->it_nred, b->x32, b->d_act, b->V, b->H, b->cs, b->sn,
                          b->g, b->y, b->h, b->res, b->part, b->nrm, b->hn, b->bn, b->dpart,
                          b->d_k};
  for (auto& gp : b->groups) {
    p.push_back(gp.m2l);
    p.push_back(gp.m2lt32);
    p.push_back(gp.m2lf);
    p.push_back(gp.m2lh);
    p.push_back(gp.m2lt);
    p.push_back(gp.cx);
    p.push_back(gp.bx);
    p.push_back(gp.nr);
  }
  for (void* q : p)
    if (q) hipFree(q);
  for (hipGraphExec_t ge : b->graph)
    if (ge) hipGraphExecDestroy(ge);
  if (b->h_pinned) hipHostFree(b->h_pinned);
  for (hipEvent_t e : b->ev)
    if (e) hipEventDestroy(e);
  if (b->own_stream) hipStreamDestroy(b->stream);
  delete b;
  return GRT_OK;
}

const char* grt_batch_error_message(const grt_batch* b) {
  return b ? b->err.c_str() : "null batch";
}

grt_status grt_batch_solve(grt_batch* b, const grt_solve_opts* o, void* const* beta,
                           grt_solve_stats* stats) {
  if (!b || !o || !beta) return GRT_EINVAL;
  b->err.clear();
  if (o->precision != GRT_FP64 && o->precision != GRT_FP32 && o->precision != GRT_FP32_RELAXED)
    return bset(b, GRT_EINVAL, "precision must be GRT_FP64, GRT_FP32 or GRT_FP32_RELAXED");
  if (!(o->tol > 0 && o->tol < 1)) return bset(b, GRT_EINVAL, "tol must be in (0, 1)");
  for (int i = 0; i < b->B; ++i)
    if (b->ctx[i]->gen != b->gen[i])
      return bset(b, GRT_ESTATE, "context " + std::to_string(i) +
                                     " changed (problem, build or table) since the batch was made");
  BHIP(b, hipSetDevice(b->device));
  auto t0 = std::chrono::steady_clock::now();
  const int m = std::max(1, std::min(o->restart > 0 ? o->restart : 100, 1000));
  const int maxit = o->maxit > 0 ? o->maxit : 1000;
  const double tol = o->tol;
  BTRY(batch_workspace(b, m));
  hipStream_t s = b->stream;
  const int B = b->B;
  const size_t ldv = (size_t)b->ntot;
  const unsigned gn = (unsigned)((b->ntot + BT - 1) / BT);
  cd* X = b->V + (size_t)(m + 1) * ldv;   // iterate (normalised)
  cd* Bv = b->V + (size_t)(m + 2) * ldv;  // right-hand side (normalised)
  const bool use_graph = o->use_graph != 0;
  // x0 and b
  BTRY(batch_rhs_hat(b, Bv));
  BHIP(b, hipMemsetAsync(X, 0, sizeof(cd) * ldv, s));
  if (o->use_x0) {
    for (int i = 0; i < B; ++i) {
      const InstDesc& q = b->hd[i];
      BHIP(b, hipMemcpyAsync(X + q.off, beta[i], sizeof(cd) * q.nbeta, hipMemcpyDeviceToDevice, s));
    }
    ew_scale_kernel<<<gn, BT, 0, s>>>(X, b->d_dnorm, X, b->ntot);
  }
  LockstepResult r(B);
  std::vector<int> refine(B, 0);
  int fast_steps = 0;
  if (o->precision == GRT_FP64 || o->precision == GRT_FP32_RELAXED) {
    const double sw = o->precision == GRT_FP64 ? 0.0
                      : o->inner_tol > 0      ? o->inner_tol
                                              : std::min(1e-2, 1e5 * tol);
    BTRY(batch_gmres(b, false, Bv, X, tol, maxit, m, o->use_x0 != 0, use_graph, r, sw,
                     &fast_steps));
  } else {
    // FP64 iterative refinement around the mixed-precision operator, for all
    // problems in lockstep: R = B - K X (FP64), solve K32 E = R to inner_tol, X += E.
    // A problem whose FP64 residual meets tol gets R = 0, so the inner solve leaves
    // it alone.
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-5;
    const int max_ref = o->max_refine > 0 ? o->max_refine : 10;
    cd* R = b->V + (size_t)(m + 5) * ldv;
    cd* E = b->V + (size_t)(m + 6) * ldv;
    std::vector<double> bn, rn;
    BTRY(batch_norms(b, Bv, b->bn));
    BTRY(read_vec(b, b->bn, bn));
    std::vector<int> flag(B, 0);
    bool guard = o->use_x0 != 0;
    for (int outer = 0; outer <= max_ref; ++outer) {
      BTRY(batch_apply(b, X, use_graph, false));
      ew_sub_kernel<<<gn, BT, 0, s>>>(Bv, b->wout, R, b->ntot);
      BTRY(batch_norms(b, R, b->nrm));
      BTRY(read_vec(b, b->nrm, rn));
      bool any = false, reject = false;
      for (int i = 0; i < B; ++i) {
        r.rel[i] = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
        if (guard && r.rel[i] >= 1.0) {
          r.rejected[i] = 1;
          reject = true;
        }
      }
      if (guard) {
        guard = false;
        if (reject) {
          // initial guesses no better than zero are dropped (residual recomputed)
          BHIP(b, hipMemcpyAsync(b->d_k, r.rejected.data(), sizeof(int) * B,
                                 hipMemcpyHostToDevice, s));
          zero_rejected_kernel<<<b->nseg, BT, 0, s>>>(b->d_seg2inst, b->d_k, X);
          BHIP(b, hipGetLastError());
          --outer;
          continue;
        }
      }
      // a problem takes no further correction once its FP64 residual meets tol or
      // it has used its own maxit inner iterations
      int budget = 0;
      for (int i = 0; i < B; ++i) {
        flag[i] = r.rel[i] <= tol || r.iters[i] >= maxit;
        if (!flag[i]) {
          any = true;
          budget = std::max(budget, maxit - r.iters[i]);
        }
      }
      if (!any || outer == max_ref) break;
      BHIP(b, hipMemcpyAsync(b->d_k, flag.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
      zero_rejected_kernel<<<b->nseg, BT, 0, s>>>(b->d_seg2inst, b->d_k, R);
      BHIP(b, hipMemsetAsync(E, 0, sizeof(cd) * ldv, s));
      LockstepResult ri(B);
      BTRY(batch_gmres(b, true, R, E, itol, budget, m, false, use_graph, ri));
      for (int i = 0; i < B; ++i) {
        r.iters[i] += ri.iters[i];
        r.cycles[i] += ri.cycles[i];
        if (!flag[i]) refine[i] += 1;
      }
      ew_add_kernel<<<gn, BT, 0, s>>>(X, E, b->ntot);
      BHIP(b, hipGetLastError());
    }
  }
  // back to beta = D^{-1} x^, scattered to the callers' vectors
  ew_scale_kernel<<<gn, BT, 0, s>>>(X, b->d_dinv, X, b->ntot);
  for (int i = 0; i < B; ++i) {
    const InstDesc& q = b->hd[i];
    BHIP(b, hipMemcpyAsync(beta[i], X + q.off, sizeof(cd) * q.nbeta, hipMemcpyDeviceToDevice, s));
  }
  BHIP(b, hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool conv = true;
  for (int i = 0; i < B; ++i) {
    if (stats) {
      stats[i] = grt_solve_stats{};
      stats[i].iters = r.iters[i];
      stats[i].cycles = r.cycles[i];
      stats[i].rel_resid = r.rel[i];
      stats[i].seconds = secs;
      stats[i].refine_steps = refine[i];
      stats[i].x0_rejected = r.rejected[i];
      // lockstep: the relaxed switch is taken for the whole batch at once
      stats[i].fp32_applies = o->precision == GRT_FP32 ? r.iters[i] + r.cycles[i]
                                                       : std::min(fast_steps, r.iters[i]);
    }
    if (!(r.rel[i] <= tol)) conv = false;
  }
  return conv ? GRT_OK : bset(b, GRT_ENOCONV, "some problems did not reach the tolerance");
}

}  // extern "C"
