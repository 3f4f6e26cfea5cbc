// Block-level device code of the apply kernels, shared by the single-problem
// launches (apply.hip) and the batched launches (batch.hip).  Each *_block
// function is the body of one workgroup; its block coordinates are parameters so
// that a batched launch can map a work item (problem, block x, block y) onto it.
#pragma once
#include "dev_bessel.h"
#include "grt_internal.h"

namespace grt {

constexpr int M2L_WAVES = 4;     // waves per block: same 64 targets, sources split 4 ways
constexpr int M2L_THREADS = 64 * M2L_WAVES;
constexpr int M2L_TILE = 16;     // sources staged in LDS at a time, per wave
constexpr int M2L_QB = 4;        // generator orders produced per block of the contraction
#ifndef M2L_HALF_MINW
#define M2L_HALF_MINW 2  // waves per SIMD asked of the register allocator for the split
                         // (half-output) translation kernels
#endif
#ifndef M2L_TNUG
#define M2L_TNUG 2               // coefficients read ahead in the table kernel's contraction
#endif
#ifndef M2L_TDIST
#define M2L_TDIST 2              // blocks of table orders in flight in the table kernel
#endif

__device__ inline __attribute__((always_inline)) void cmac(cf& acc, cf a, cf b) {
  acc.r = fmaf(a.r, b.r, acc.r);
  acc.r = fmaf(-a.i, b.i, acc.r);
  acc.i = fmaf(a.r, b.i, acc.i);
  acc.i = fmaf(a.i, b.r, acc.i);
}
__device__ inline cd to_acc(cd v, cd*) { return v; }
__device__ inline cf to_acc(cd v, cf*) { return cf{(float)v.r, (float)v.i}; }

// Toeplitz generator of one (target, source) pair, FP64:
//   tau_q = sum_l alpha^l H_q(k rho_l) e^{i q phi_l},  rho_l e^{i phi_l} = (dx - l d) + i dy,
// for the copies l = -1, 0, 1 (Graf's theorem for each copy), q = -2P..2P.  H_0, H_1
// come from the table, H_q from the upward recurrence and e^{i q phi} from powers.
// emit0(tau_0) is called first, then emit(qb, tp, tm) for each block of M2L_QB
// orders with tp[u] = tau_q, tm[u] = tau_{-q}, q = 1 + qb M2L_QB + u (zero past 2P).
// skip0 drops the copy l = 0 (the excluded self term); dead drops everything; with
// zsafe > 0 the pair is dropped too when a kept copy has k rho < zsafe.  MID_ONLY:
// only the copy l = 0 (weight wl[1]) is generated.
template <int P, typename TabPtr, typename F0, typename F, bool MID_ONLY = false>
__device__ __forceinline__ void pair_generate(double dx, double dy, double k, double d,
                                              const cd* wl, bool skip0, bool dead, TabPtr tab,
                                              double zsafe, F0&& emit0, F&& emit) {
  constexpr int NQB = (2 * P + M2L_QB - 1) / M2L_QB;
  constexpr int L0 = MID_ONLY ? 1 : 0, L1 = MID_ONLY ? 2 : 3;
  cd hp[3], hc[3], cc[3], cq[3];
  double rz2[3];
  double zz[3];
  bool near = false;
#pragma unroll
  for (int l = L0; l < L1; ++l) {
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
  for (int l = L0; l < L1; ++l) {
    bool off = (skip0 && l == 1) || dead || near;
    cd h0, h1;
    hankel01_tab(zz[l], tab, h0, h1);
    cd w = off ? cd{0.0, 0.0} : wl[l];
    hp[l] = w * h0;
    hc[l] = w * h1;
  }
  if constexpr (MID_ONLY)
    emit0(hp[1]);
  else
    emit0(hp[0] + hp[1] + hp[2]);
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    cd tp[M2L_QB], tm[M2L_QB];
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      cd sp{0.0, 0.0}, sm{0.0, 0.0};
      if (q <= 2 * P) {
#pragma unroll
        for (int l = L0; l < L1; ++l) {
          // sp += hc cq, sm += hc conj(cq), as FMAs
          sp.r = fma(hc[l].r, cq[l].r, sp.r);
          sp.r = fma(-hc[l].i, cq[l].i, sp.r);
          sp.i = fma(hc[l].r, cq[l].i, sp.i);
          sp.i = fma(hc[l].i, cq[l].r, sp.i);
          sm.r = fma(hc[l].r, cq[l].r, sm.r);
          sm.r = fma(hc[l].i, cq[l].i, sm.r);
          sm.i = fma(hc[l].i, cq[l].r, sm.i);
          sm.i = fma(-hc[l].r, cq[l].i, sm.i);
        }
        if (q & 1) sm = -sm;  // H_{-q} = (-1)^q H_q
        if (q < 2 * P) {
#pragma unroll
          for (int l = L0; l < L1; ++l) {
            cd hn = (q * rz2[l]) * hc[l] - hp[l];
            hp[l] = hc[l];
            hc[l] = hn;
            cq[l] = cq[l] * cc[l];
          }
        }
      }
      tp[u] = sp;
      tm[u] = sm;
    }
    emit(qb, tp, tm);
  }
}

// acc[n - LO] += sum over the block's orders q of tau_q x[n+q] + tau_{-q} x[n-q] for
// the outputs n in [LO, LO + NH) (n = -P..P at index n + P; by default all of them);
// each x[nu] is read once per block and feeds up to 2 M2L_QB complex FMAs.
template <int P, typename T, typename BP, int NUG = 1 << 20, int LO = 0, int NH = 2 * P + 1>
__device__ __forceinline__ void contract_block(T* acc, BP b, int qb, const T* tp, const T* tm) {
  constexpr int NB = 2 * P + 1;
  // x may be re-read here: keeps x[nu] out of registers across blocks of orders
  asm volatile("" ::: "memory");
#pragma unroll
  for (int nu = 0; nu < NB; ++nu) {
    bool need = false;
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      if (q <= 2 * P && ((nu - q >= LO && nu - q < LO + NH) || (nu + q >= LO && nu + q < LO + NH)))
        need = true;
    }
    if (!need) continue;
    const T bv = b[nu];
    // with NUG set, at most NUG coefficients are read ahead of their use
    if (nu % NUG == NUG - 1) asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      if (q > 2 * P) continue;
      if (nu - q >= LO && nu - q < LO + NH) cmac(acc[nu - q - LO], tp[u], bv);  // t_q x[n+q]
      if (nu + q >= LO && nu + q < LO + NH) cmac(acc[nu + q - LO], tm[u], bv);  // t_{-q} x[n-q]
    }
  }
}

// Contribution of one source inclusion (and its copies) to the incoming
// coefficients acc[n - LO] of one target, n in [LO, LO + NH): acc[n] += sum_nu
// tau_{nu-n} x[nu], with the generator computed on the fly.  T is the accumulation
// type (cd: FP64, cf: FP32 with FP32 accumulation; the generator is FP64 either way).
template <int P, typename T, typename BP, typename TabPtr, int LO = 0, int NH = 2 * P + 1,
          bool MID_ONLY = false>
__device__ __forceinline__ void pair_accumulate(T* acc, BP b, double dx, double dy, double k,
                                                double d, const cd* wl, bool skip0, bool dead,
                                                TabPtr tab, double zsafe) {
  auto e0 = [&](cd t0) {
    const T t = to_acc(t0, (T*)nullptr);
#pragma unroll
    for (int n = 0; n < NH; ++n) cmac(acc[n], t, b[n + LO]);
  };
  auto e1 = [&](int qb, const cd* tp, const cd* tm) {
    T a[M2L_QB], c[M2L_QB];
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      a[u] = to_acc(tp[u], (T*)nullptr);
      c[u] = to_acc(tm[u], (T*)nullptr);
    }
    contract_block<P, T, BP, 1 << 20, LO, NH>(acc, b, qb, a, c);
  };
  pair_generate<P, TabPtr, decltype(e0)&, decltype(e1)&, MID_ONLY>(dx, dy, k, d, wl, skip0, dead,
                                                                   tab, zsafe, e0, e1);
}

// Translation of the outgoing coefficients of sources [m0, m1) (and of their
// copies l = -1, 0, 1) into incoming coefficients at 64 targets (one per lane);
// the block's four waves take a quarter of the sources each, stage them in LDS
// (every lane then reads the same address: a broadcast) and are summed through
// LDS at the end.  T = cd: FP64; T = cf: FP32 contraction and accumulation with
// pairs closer than zsafe left out.  Only the outputs n in [LO, LO + NH) (index
// n + P) are formed and stored: a launch may split them over two blocks, each
// recomputing the generator, to halve the accumulators a lane holds.
template <int P, typename T, int LO = 0, int NH = 2 * P + 1>
__device__ __forceinline__ void m2l_block(const double* __restrict__ cx,
                                                          const double* __restrict__ cy,
                                                          const T* __restrict__ x, T* partial,
                                                          int M, int chunk, double k, double d,
                                                          cd alpha, cd alpha_inv,
                                                          const double* __restrict__ htab,
                                                          double zsafe, int bx_, int by_) {
  constexpr int NB = 2 * P + 1;
  constexpr int TW = sizeof(T) / sizeof(double);  // doubles per complex value (1 or 2)
  constexpr int STAGE = M2L_WAVES * M2L_TILE * (TW * NB + 2);
  constexpr int RED = TW * NH * 64;
  constexpr int BUF = STAGE > RED ? STAGE : RED;
  __shared__ double smem[BUF];
  __shared__ double stab[HTAB_SIZE];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  T* sx = reinterpret_cast<T*>(smem) + wv * M2L_TILE * NB;
  double* scx = smem + TW * M2L_WAVES * M2L_TILE * NB + wv * 2 * M2L_TILE;
  double* scy = scx + M2L_TILE;
  const int j = bx_ * 64 + lane;
  const int m0 = by_ * chunk;
  const int m1 = min(M, m0 + chunk);
  const int per = (m1 - m0 + M2L_WAVES - 1) / M2L_WAVES;
  const int s0 = m0 + wv * per;
  const int s1 = min(m1, s0 + per);
  const int ntile = (per + M2L_TILE - 1) / M2L_TILE;  // same for every wave: barriers match
  for (int t = threadIdx.x; t < HTAB_SIZE; t += M2L_THREADS) stab[t] = htab[t];
  const bool live = j < M;
  const double xj = live ? cx[j] : 0.0, yj = live ? cy[j] : 0.0;
  T acc[NH];
#pragma unroll
  for (int n = 0; n < NH; ++n) acc[n] = T{0, 0};
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
      pair_accumulate<P, T, const T*, const double*, LO, NH>(
          acc, sx + mm * NB, xj - scx[mm], yj - scy[mm], k, d, wl, j == m, !live, stab, zsafe);
    }
  }
  // sum the four waves' partial results through LDS: wave 3, then 2, then 1 add into
  // the buffer in turn, wave 0 adds its own and stores
  T* red = reinterpret_cast<T*>(smem);
  for (int src = M2L_WAVES - 1; src >= 1; --src) {
    __syncthreads();
    if (wv == src) {
#pragma unroll
      for (int n = 0; n < NH; ++n) {
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
    T* out = partial + ((size_t)by_ * M + j) * NB + LO;
#pragma unroll
    for (int n = 0; n < NH; ++n) {
      T o = red[n * 64 + lane];
      out[n] = T{acc[n].r + o.r, acc[n].i + o.i};
    }
  }
}

// ---------------------------------------------------------------------------
// Resident translation table.  The generator tau^{(jm)} does not depend on the
// coefficients, so for one geometry it can be built once and streamed by every
// apply: table[(m NQ + q + 2P) Mpad + j] = tau_q of target j, source m, NQ = 4P+1,
// Mpad = M rounded up to 64 (zero rows for j >= M).  Consecutive targets are
// consecutive in memory, so the 64 lanes of a wave read one 1 KB line per order.
// ---------------------------------------------------------------------------

// One lane per target, sources [by_ chunk, (by_+1) chunk).  T = cd: the FP64 table
// of every pair; T = cf with zsafe > 0: the FP32 table of the mixed-precision apply,
// whose near pairs (a kept copy at k rho < zsafe, done in FP64 elsewhere) are zero.
template <int P, typename T = cd>
__device__ __forceinline__ void table_build_block(const double* __restrict__ cx,
                                                  const double* __restrict__ cy, int M, int Mpad,
                                                  int chunk, double k, double d, cd alpha,
                                                  cd alpha_inv, const double* __restrict__ htab,
                                                  T* table, int bx_, int by_,
                                                  double zsafe = 0.0) {
  constexpr int NQ = 4 * P + 1;
  __shared__ double stab[HTAB_SIZE];
  for (int t = threadIdx.x; t < HTAB_SIZE; t += blockDim.x) stab[t] = htab[t];
  __syncthreads();
  const int j = bx_ * 64 + (threadIdx.x & 63);
  if (j >= M) return;
  const int m0 = by_ * chunk, m1 = min(M, m0 + chunk);
  const double xj = cx[j], yj = cy[j];
  const cd wl[3] = {alpha_inv, cd{1.0, 0.0}, alpha};
  for (int m = m0; m < m1; ++m) {
    T* col = table + (size_t)m * NQ * Mpad + j;
    pair_generate<P>(
        xj - cx[m], yj - cy[m], k, d, wl, j == m, false, stab, zsafe,
        [&](cd t0) { col[(size_t)(2 * P) * Mpad] = to_acc(t0, (T*)nullptr); },
        [&](int qb, const cd* tp, const cd* tm) {
#pragma unroll
          for (int u = 0; u < M2L_QB; ++u) {
            const int q = 1 + qb * M2L_QB + u;
            if (q > 2 * P) continue;
            col[(size_t)(2 * P + q) * Mpad] = to_acc(tp[u], (T*)nullptr);
            col[(size_t)(2 * P - q) * Mpad] = to_acc(tm[u], (T*)nullptr);
          }
        });
  }
}

// Streaming read of one table entry: each entry is used exactly once per apply, so
// it is loaded non-temporally (it should not displace the reused data in the caches).
__device__ __forceinline__ cd ld_stream(const cd* p) {
  return cd{__builtin_nontemporal_load(&p->r), __builtin_nontemporal_load(&p->i)};
}
__device__ __forceinline__ cf ld_stream(const cf* p) {
  return cf{__builtin_nontemporal_load(&p->r), __builtin_nontemporal_load(&p->i)};
}

// Same result as m2l_block, with the generator read from the resident table (the
// next block of orders is loaded while the current one is contracted).  T = cd: the
// FP64 apply; T = cf: the FP32 table, coefficients and accumulation of the
// mixed-precision apply (near pairs are zero in that table).
template <int P, typename T = cd>
__device__ __forceinline__ void m2l_table_block(const T* __restrict__ table,
                                                const T* __restrict__ x, T* partial, int M,
                                                int Mpad, int chunk, int bx_, int by_) {
  constexpr int NB = 2 * P + 1;
  constexpr int NQ = 4 * P + 1;
  constexpr int NQB = (2 * P + M2L_QB - 1) / M2L_QB;
  constexpr int TW = sizeof(T) / sizeof(double);  // doubles per complex value (1 or 2)
  constexpr int STAGE = TW * M2L_WAVES * M2L_TILE * NB;
  constexpr int RED = TW * NB * 64;
  constexpr int BUF = STAGE > RED ? STAGE : RED;
  __shared__ double smem[BUF];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  T* sx = reinterpret_cast<T*>(smem) + wv * M2L_TILE * NB;
  const int j = bx_ * 64 + lane;  // < Mpad: table rows of dead lanes are zero
  const int m0 = by_ * chunk;
  const int m1 = min(M, m0 + chunk);
  const int per = (m1 - m0 + M2L_WAVES - 1) / M2L_WAVES;
  const int s0 = m0 + wv * per;
  const int s1 = min(m1, s0 + per);
  const int ntile = (per + M2L_TILE - 1) / M2L_TILE;
  T acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = T{0, 0};
  // table row of order q for source m: a wave-uniform base plus the lane's target
  auto row = [&](const T* col, int q) { return ld_stream(col + (size_t)(2 * P + q) * Mpad + j); };
  for (int it = 0; it < ntile; ++it) {
    const int ts = s0 + it * M2L_TILE;
    const int cnt = max(0, min(M2L_TILE, s1 - ts));
    __syncthreads();
    for (int t = lane; t < cnt * NB; t += 64) sx[t] = x[(size_t)ts * NB + t];
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      const T* b = sx + mm * NB;
      const T* col = table + (size_t)(ts + mm) * NQ * Mpad;
      {
        const T t0 = row(col, 0);
#pragma unroll
        for (int n = 0; n < NB; ++n) cmac(acc[n], t0, b[n]);
      }
      // blocks of orders in flight: the current one and the next M2L_TDIST - 1
      T np[M2L_TDIST][M2L_QB], nm[M2L_TDIST][M2L_QB];
#pragma unroll
      for (int d = 0; d < M2L_TDIST; ++d)
#pragma unroll
        for (int u = 0; u < M2L_QB; ++u) {
          const int q = 1 + d * M2L_QB + u;
          np[d][u] = q <= 2 * P ? row(col, q) : T{0, 0};
          nm[d][u] = q <= 2 * P ? row(col, -q) : T{0, 0};
        }
#pragma unroll
      for (int qb = 0; qb < NQB; ++qb) {
        constexpr int D = M2L_TDIST;
        T tp[M2L_QB], tm[M2L_QB];
#pragma unroll
        for (int u = 0; u < M2L_QB; ++u) {
          tp[u] = np[qb % D][u];
          tm[u] = nm[qb % D][u];
        }
        if (qb + D < NQB) {
#pragma unroll
          for (int u = 0; u < M2L_QB; ++u) {
            const int q = 1 + (qb + D) * M2L_QB + u;
            np[qb % D][u] = q <= 2 * P ? row(col, q) : T{0, 0};
            nm[qb % D][u] = q <= 2 * P ? row(col, -q) : T{0, 0};
          }
        }
        contract_block<P, T, const T*, M2L_TNUG>(acc, b, qb, tp, tm);
      }
    }
  }
  T* red = reinterpret_cast<T*>(smem);
  for (int src = M2L_WAVES - 1; src >= 1; --src) {
    __syncthreads();
    if (wv == src) {
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        T v = acc[n];
        if (src != M2L_WAVES - 1) {
          const T o = red[n * 64 + lane];
          v.r += o.r;
          v.i += o.i;
        }
        red[n * 64 + lane] = v;
      }
    }
  }
  __syncthreads();
  if (wv == 0 && j < M) {
    T* out = partial + ((size_t)by_ * M + j) * NB;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const T o = red[n * 64 + lane];
      out[n] = T{acc[n].r + o.r, acc[n].i + o.i};
    }
  }
}

// Half contraction for the two-lanes-per-target table kernel: outputs n = -P..0
// only (local index 0..P), acc[n] += sum over the block's orders of
// tau_q x[n+q] + tau_{-q} x[n-q].
constexpr int NU_GROUP = 2;  // coefficients read from LDS per group in the half contraction
constexpr int T2_TILE = 8;   // sources staged per wave in the two-lanes table kernel
template <int P, typename BP>
__device__ __forceinline__ void contract_block_half(cd* acc, BP b, int qb, const cd* tp,
                                                    const cd* tm) {
  constexpr int NB = 2 * P + 1;
  constexpr int NH = P + 1;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int nu = 0; nu < NB; ++nu) {
    bool need = false;
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      if (q <= 2 * P && ((nu - q >= 0 && nu - q < NH) || nu + q < NH)) need = true;
    }
    if (!need) continue;
    const cd bv = b[nu];
    // a few coefficients in flight at a time: the LDS reads are not all hoisted
    if (nu % NU_GROUP == NU_GROUP - 1) asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < M2L_QB; ++u) {
      const int q = 1 + qb * M2L_QB + u;
      if (q > 2 * P) continue;
      if (nu - q >= 0 && nu - q < NH) cmac(acc[nu - q], tp[u], bv);
      if (nu + q < NH) cmac(acc[nu + q], tm[u], bv);
    }
  }
}

// Resident-table translation with two lanes per target.  The Toeplitz contraction
// is symmetric under reflection: with tau'_q = tau_{-q} and x'[nu] = x[-nu], the
// outputs n = 0..P equal the outputs -n of the same contraction on (tau', x').  So
// lane 2i computes n = -P..0 of target i and lane 2i+1 the same formula on the
// reflected table entries and coefficients (lane-dependent addresses, identical
// instructions), each holding P+1 accumulators instead of 2P+1; the two lanes read
// the same table lines.  32 targets per wave, four waves splitting the sources.
template <int P>
__device__ __forceinline__ void m2l_table2_block(const cd* __restrict__ table,
                                                 const cd* __restrict__ x, cd* partial, int M,
                                                 int Mpad, int chunk, int bx_, int by_) {
  constexpr int NB = 2 * P + 1;
  constexpr int NH = P + 1;
  constexpr int NQ = 4 * P + 1;
  constexpr int NQB = (2 * P + M2L_QB - 1) / M2L_QB;
  constexpr int STAGE = 2 * M2L_WAVES * T2_TILE * 2 * NB;  // forward and reflected copies
  constexpr int RED = 2 * NH * 64;
  constexpr int BUF = STAGE > RED ? STAGE : RED;
  __shared__ double smem[BUF];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const bool h = lane & 1;                // 0: n = -P..0, 1: n = 0..P (reflected)
  cd* sx = reinterpret_cast<cd*>(smem) + wv * T2_TILE * 2 * NB;
  const int j = bx_ * 32 + (lane >> 1);  // < Mpad: table rows of dead targets are zero
  const int m0 = by_ * chunk;
  const int m1 = min(M, m0 + chunk);
  const int per = (m1 - m0 + M2L_WAVES - 1) / M2L_WAVES;
  const int s0 = m0 + wv * per;
  const int s1 = min(m1, s0 + per);
  const int ntile = (per + T2_TILE - 1) / T2_TILE;
  cd acc[NH];
#pragma unroll
  for (int n = 0; n < NH; ++n) acc[n] = cd{0, 0};
  for (int it = 0; it < ntile; ++it) {
    const int ts = s0 + it * T2_TILE;
    const int cnt = max(0, min(T2_TILE, s1 - ts));
    __syncthreads();
    // each source staged forwards (x[nu], even lanes) and reflected (x[NB-1-nu], odd
    // lanes), so every lane reads at constant offsets from its own base
    for (int t = lane; t < cnt * NB; t += 64) {
      const int mm = t / NB, nu = t - mm * NB;
      const cd v = x[(size_t)ts * NB + t];
      sx[mm * 2 * NB + nu] = v;
      sx[mm * 2 * NB + NB + (NB - 1 - nu)] = v;
    }
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      const cd* b = sx + mm * 2 * NB + h * NB;
      // both lanes of a target load the same two rows (+q, -q): row offsets are
      // wave-uniform, and the odd lane swaps their roles
      const cd* col = table + (size_t)(ts + mm) * NQ * Mpad;
      {
        const cd t0 = ld_stream(col + (size_t)(2 * P) * Mpad + j);
#pragma unroll
        for (int n = 0; n < NH; ++n) cmac(acc[n], t0, b[n]);
      }
      cd np[M2L_QB], nm[M2L_QB];
#pragma unroll
      for (int u = 0; u < M2L_QB; ++u) {
        const int q = 1 + u;
        np[u] = q <= 2 * P ? ld_stream(col + (size_t)(2 * P + q) * Mpad + j) : cd{0, 0};
        nm[u] = q <= 2 * P ? ld_stream(col + (size_t)(2 * P - q) * Mpad + j) : cd{0, 0};
      }
#pragma unroll
      for (int qb = 0; qb < NQB; ++qb) {
        cd tp[M2L_QB], tm[M2L_QB];
#pragma unroll
        for (int u = 0; u < M2L_QB; ++u) {
          tp[u] = h ? nm[u] : np[u];
          tm[u] = h ? np[u] : nm[u];
        }
        if (qb + 1 < NQB) {
#pragma unroll
          for (int u = 0; u < M2L_QB; ++u) {
            const int q = 1 + (qb + 1) * M2L_QB + u;
            np[u] = q <= 2 * P ? ld_stream(col + (size_t)(2 * P + q) * Mpad + j) : cd{0, 0};
            nm[u] = q <= 2 * P ? ld_stream(col + (size_t)(2 * P - q) * Mpad + j) : cd{0, 0};
          }
        }
        contract_block_half<P, const cd*>(acc, b, qb, tp, tm);
      }
    }
  }
  cd* red = reinterpret_cast<cd*>(smem);
  for (int src = M2L_WAVES - 1; src >= 1; --src) {
    __syncthreads();
    if (wv == src) {
#pragma unroll
      for (int n = 0; n < NH; ++n) {
        cd v = acc[n];
        if (src != M2L_WAVES - 1) v += red[n * 64 + lane];
        red[n * 64 + lane] = v;
      }
    }
  }
  __syncthreads();
  if (wv == 0 && j < M) {
    cd* out = partial + ((size_t)by_ * M + j) * NB;
#pragma unroll
    for (int n = 0; n < NH; ++n) {
      const cd v = acc[n] + red[n * 64 + lane];
      // even lane: n - P in -P..0; odd lane: -(n - P) in 0..P (its n = P is 0: skipped)
      if (h == 0)
        out[n] = v;
      else if (n < P)
        out[2 * P - n] = v;
    }
  }
}

// FP64 translation over the near pairs (the pairs the FP32 pass leaves out): one
// lane per pair (target ntgt[e], source nlist[e]); each pair's contribution goes to
// its own row of part, summed per target in list order by near_reduce_kernel.
// One near pair e of the CSR list (target ntgt[e], source nlist[e]) in FP64:
// part[e][n] = sum over the three copies of T(j <- m) x_m (stab: the H_0/H_1 table,
// already in LDS).
template <int P>
__device__ __forceinline__ void near_pair(const double* __restrict__ cx,
                                          const double* __restrict__ cy,
                                          const cd* __restrict__ x, const int* __restrict__ ntgt,
                                          const int* __restrict__ nlist, cd* part, int e,
                                          double k, double d, cd alpha, cd alpha_inv,
                                          const double* stab) {
  constexpr int NB = 2 * P + 1;
  const int j = ntgt[e], m = nlist[e];
  cd acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = cd{0.0, 0.0};
  const cd wl[3] = {alpha_inv, cd{1.0, 0.0}, alpha};
  pair_accumulate<P, cd>(acc, x + (size_t)m * NB, cx[j] - cx[m], cy[j] - cy[m], k, d, wl, j == m,
                         false, stab, 0.0);
  cd* o = part + (size_t)e * NB;
#pragma unroll
  for (int n = 0; n < NB; ++n) o[n] = acc[n];
}

template <int P>
__global__ void __launch_bounds__(64) m2l_near_kernel(const double* __restrict__ cx,
                                                      const double* __restrict__ cy,
                                                      const cd* __restrict__ x,
                                                      const int* __restrict__ ntgt,
                                                      const int* __restrict__ nlist, cd* part,
                                                      int npairs, double k, double d, cd alpha,
                                                      cd alpha_inv,
                                                      const double* __restrict__ htab) {
  __shared__ double stab[HTAB_SIZE];
  for (int t = threadIdx.x; t < HTAB_SIZE; t += 64) stab[t] = htab[t];
  __syncthreads();
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e < npairs) near_pair<P>(cx, cy, x, ntgt, nlist, part, e, k, d, alpha, alpha_inv, stab);
}

// out[idx] for idx = j NB + n: the sum over the near pairs of target j (CSR order) of
// part[e][n]
__device__ __forceinline__ void near_reduce_entry(const int* __restrict__ noff,
                                                  const cd* __restrict__ part, int NB, cd* out,
                                                  int idx) {
  const int j = idx / NB, n = idx - j * NB;
  cd s{0, 0};
  for (int e = noff[j]; e < noff[j + 1]; ++e) s += part[(size_t)e * NB + n];
  out[idx] = s;
}

static __global__ void near_reduce_kernel(const int* __restrict__ noff, const cd* __restrict__ part,
                                          int M, int NB, cd* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < M * NB) near_reduce_entry(noff, part, NB, out, idx);
}

constexpr int CX_WAVES = 4;   // waves per block: same 64 targets, sources split 4 ways
constexpr int CX_TUNE_MIN_PER = 1;  // fewest sources per wave among the tuner's candidates
constexpr int BX_TUNE_MIN_PER = 2;
constexpr int CX_TUNE_MAX_CHUNKS = 1024;  // most partial results among the candidates
constexpr int BX_TUNE_MAX_CHUNKS = 128;
constexpr int CX_TILE = 8;    // inclusions staged in LDS at a time, per wave

// Field of all multipoles (and their copies) at the C targets, one per lane:
//   target t < N: Gamma_1 node, t < 2N: Gamma_2 node (value, normal derivative over
//   3 copies),
//   t < 2N + Nw2: middle wall node (value, d/dx, cancelled two-term form
//   alpha^2 Phi(L-d) - alpha^{-1} Phi(L+2d), Phi the l = 0 field).
// With F_n = H_n(k r) e^{in theta}: value = sum x[n] F_n and, by
// (d_x +- i d_y) F_n = -+ k F_{n+-1}, d/dx = (k/2)(A - B), d/dy = (ik/2)(A + B)
// with A = sum x[n] F_{n-1}, B = sum x[n] F_{n+1}.
// partial[chunk][t][0..1] = (value, derivative) over the chunk's inclusions.  A block
// has CX_WAVES waves on the same 64 targets, each taking a share of the chunk's
// sources; the H_0/H_1 table is staged once per block and the waves' sums are added
// through LDS in a fixed order.
template <int P>
__device__ __forceinline__ void cx_block(const DevGeom& g, const double* __restrict__ cx,
                                         const double* __restrict__ cy,
                                         const cd* __restrict__ x, cd* partial, int chunk,
                                         const double* __restrict__ htab, int bx_, int by_) {
  constexpr int NB = 2 * P + 1;
  __shared__ cd sx_all[CX_WAVES * CX_TILE * NB];
  __shared__ double sc_all[CX_WAVES * 2 * CX_TILE];
  __shared__ double stab[HTAB_SIZE];
  __shared__ cd red[CX_WAVES * 64 * 3];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  cd* sx = sx_all + wv * CX_TILE * NB;
  double* scx = sc_all + wv * 2 * CX_TILE;
  double* scy = scx + CX_TILE;
  const int nt = 2 * g.N + g.Nw[1];
  const int t = bx_ * 64 + lane;
  const int c0 = by_ * chunk;
  const int c1 = min(g.M, c0 + chunk);
  const int per = (c1 - c0 + CX_WAVES - 1) / CX_WAVES;
  const int m0 = c0 + wv * per;
  const int m1 = min(c1, m0 + per);
  const int ntile = (per + CX_TILE - 1) / CX_TILE;  // same for every wave: barriers match
  for (int i = threadIdx.x; i < HTAB_SIZE; i += blockDim.x) stab[i] = htab[i];
  const bool live = t < nt;
  const int tt = live ? t : 0;
  double tx[3], ty;
  cd w[3];
  const bool wall = tt >= 2 * g.N;
  double tnx = 0.0, tny = 1.0;  // the interface's normal at the target
  if (!wall) {
    const double* nd = g.node + (size_t)tt * NODE_STRIDE;  // Gamma_1 nodes, then Gamma_2
    const double x0 = nd[0];
    ty = nd[1];
    tnx = nd[2];
    tny = nd[3];
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
  if (wall) w[2] = cd{0.0, 0.0};  // two-term form: the third position is not used
  const double k = g.k[1];
  cd val{0, 0}, A{0, 0}, B{0, 0};
  for (int it = 0; it < ntile; ++it) {
    const int ts = m0 + it * CX_TILE;
    const int cnt = max(0, min(CX_TILE, m1 - ts));
    __syncthreads();
    for (int i = lane; i < cnt * NB; i += 64) sx[i] = x[(size_t)ts * NB + i];
    for (int i = lane; i < cnt; i += 64) {
      scx[i] = cx[ts + i];
      scy[i] = cy[ts + i];
    }
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      const cd* b = sx + mm * NB;
      // the copies' (or wall terms') weights are folded into H_0, H_1, so one sum
      // F_n = sum_im w_im H_n(k r_im) e^{i n theta_im} serves all three positions
      cd hp[3], hc[3], e[3], ep[3];
      double rz2[3];
#pragma unroll
      for (int im = 0; im < 3; ++im) {
        const double vx = tx[im] - scx[mm], vy = ty - scy[mm];
        const double r = sqrt(vx * vx + vy * vy);
        const double z = k * r;
        const double ir = 1.0 / r;
        e[im] = cd{vx * ir, vy * ir};
        ep[im] = e[im];
        rz2[im] = 2.0 / z;
        cd h0, h1;
        hankel01_tab(z, stab, h0, h1);
        hp[im] = w[im] * h0;
        hc[im] = w[im] * h1;
      }
      const cd F0 = hp[0] + hp[1] + hp[2];
      cmac(val, F0, b[P]);
      if (P >= 1) {
        cmac(A, F0, b[P + 1]);
        cmac(B, F0, b[P - 1]);
      }
#pragma unroll
      for (int mo = 1; mo <= P + 1; ++mo) {
        cd Fp{0, 0}, Fm{0, 0};  // F_mo and F_{-mo} = (-1)^mo sum H_mo e^{-i mo theta}
#pragma unroll
        for (int im = 0; im < 3; ++im) {
          Fp.r = fma(hc[im].r, ep[im].r, Fp.r);
          Fp.r = fma(-hc[im].i, ep[im].i, Fp.r);
          Fp.i = fma(hc[im].r, ep[im].i, Fp.i);
          Fp.i = fma(hc[im].i, ep[im].r, Fp.i);
          Fm.r = fma(hc[im].r, ep[im].r, Fm.r);
          Fm.r = fma(hc[im].i, ep[im].i, Fm.r);
          Fm.i = fma(hc[im].i, ep[im].r, Fm.i);
          Fm.i = fma(-hc[im].r, ep[im].i, Fm.i);
        }
        if (mo & 1) Fm = -Fm;
        if (mo <= P) {
          cmac(val, Fp, b[P + mo]);
          cmac(val, Fm, b[P - mo]);
        }
        if (mo + 1 <= P) cmac(A, Fp, b[P + mo + 1]);
        if (1 - mo >= -P) cmac(A, Fm, b[P + 1 - mo]);
        if (mo - 1 <= P) cmac(B, Fp, b[P + mo - 1]);
        if (-mo - 1 >= -P) cmac(B, Fm, b[P - mo - 1]);
        if (mo <= P) {
#pragma unroll
          for (int im = 0; im < 3; ++im) {
            const cd hn = (mo * rz2[im]) * hc[im] - hp[im];
            hp[im] = hc[im];
            hc[im] = hn;
            ep[im] = ep[im] * e[im];
          }
        }
      }
    }
  }
  red[(wv * 64 + lane) * 3 + 0] = val;
  red[(wv * 64 + lane) * 3 + 1] = A;
  red[(wv * 64 + lane) * 3 + 2] = B;
  __syncthreads();
  if (wv != 0 || !live) return;
  for (int v = 1; v < CX_WAVES; ++v) {
    val += red[(v * 64 + lane) * 3 + 0];
    A += red[(v * 64 + lane) * 3 + 1];
    B += red[(v * 64 + lane) * 3 + 2];
  }
  // d/dx = (k/2)(A - B), d/dy = (ik/2)(A + B); interface rows take the normal derivative
  const cd gx = (0.5 * k) * (A - B);
  cd der = wall ? gx : tnx * gx + tny * times_i((0.5 * k) * (A + B));
  cd* o = partial + ((size_t)by_ * nt + t) * 2;
  o[0] = val;
  o[1] = der;
}

// Row placement of target t's value and derivative in g: Gamma_1 (the row is
// u_1 - u_2 and the inclusions live in layer 2: minus), Gamma_2, middle wall.
__device__ __forceinline__ void cx_store(const DevGeom& g, int t, cd v, cd dv, cd* gv) {
  const int N = g.N;
  if (t < N) {
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

// The same sum with one thread per target, the chunks added in order: consecutive
// threads read consecutive partials of a chunk (coalesced).
__device__ inline void cx_reduce_rows(const DevGeom& g, const cd* partial, int nchunks, cd* gv,
                                      int t) {
  const int nt = 2 * g.N + g.Nw[1];
  if (t >= nt) return;
  cd v{0, 0}, dv{0, 0};
  // unrolled: several chunks' loads in flight, added in chunk order
#pragma unroll 8
  for (int c = 0; c < nchunks; ++c) {
    const cd* p = partial + ((size_t)c * nt + t) * 2;
    v += p[0];
    dv += p[1];
  }
  cx_store(g, t, v, dv, gv);
}

// g (rows Gamma_1 v/n, Gamma_2 v/n, wall-2 v/d) from the chunk partials: one
// wavefront per target, lanes over chunks, fixed-order tree sum.
__device__ inline void cx_reduce_block(const DevGeom& g, const cd* partial, int nchunks,
                                                        cd* gv, int bx_) {
  const int nt = 2 * g.N + g.Nw[1];
  const int t = (bx_ * blockDim.x + threadIdx.x) >> 6;
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
  cx_store(g, t, cd{vr, vi}, cd{dr, di}, gv);
}

// Incoming coefficients at inclusion j from the interface densities (P2L, Graf's
// theorem for H_0 about c_j):
//   alpha_j[n] += (i/4) w sum_l alpha^l [G^l_n sigma
//                 + (k/2)((n_x - i n_y) G^l_{n-1} - (n_x + i n_y) G^l_{n+1}) mu],
//   G^l_n = H_n(k|v_l|) e^{-in theta_l}, v_l = node + l d e_x - c_j,
// w = hs * speed the node's arc-length weight, the mu term being the derivative of
// the sigma term along the source normal n (gradient identities
// (d_x +- i d_y) G_n = +-k G_{n-+1}).  Sources: 2 interfaces x N nodes, chunked over
// blockIdx.y; the three copies of a node share its densities, so their generators
// are summed (weights alpha^l folded into H_0, H_1) before the contraction.  Each
// order m of the sum feeds acc[m] (sigma) and acc[m -+ 1] (mu).
constexpr int BX_WAVES = 4;  // waves per block: same 64 targets, nodes split 4 ways
template <int P>
__device__ __forceinline__ void bx_block(const DevGeom& g, const double* __restrict__ cx,
                                         const double* __restrict__ cy,
                                         const cd* __restrict__ w, cd* partial, int chunk,
                                         const double* __restrict__ htab, int bx_, int by_) {
  constexpr int NB = 2 * P + 1;
  __shared__ double stab[HTAB_SIZE];
  __shared__ cd red[NB * 64];
  for (int i = threadIdx.x; i < HTAB_SIZE; i += blockDim.x) stab[i] = htab[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int j = bx_ * 64 + lane;
  const int c0 = by_ * chunk;
  const int c1 = min(2 * g.N, c0 + chunk);
  const int per = (c1 - c0 + BX_WAVES - 1) / BX_WAVES;
  const int s0 = c0 + wv * per;
  const int s1 = min(c1, s0 + per);
  const bool live = j < g.M;
  const double xj = live ? cx[j] : 0.0, yj = live ? cy[j] : 0.0;
  const double k = g.k[1];
  const cd wl[3] = {g.alpha_inv, cd{1.0, 0.0}, g.alpha};
  cd acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = cd{0.0, 0.0};
  for (int sidx = s0; sidx < s1; ++sidx) {
    const int line = sidx / g.N;
    const int i = sidx - line * g.N;
    const double* nd = g.node + (size_t)sidx * NODE_STRIDE;
    const double sx0 = nd[0];
    const double syp = nd[1];
    const cd mu = w[g.col_off[line == 0 ? CB_MU1 : CB_MU2] + i];
    const cd sg = w[g.col_off[line == 0 ? CB_SIG1 : CB_SIG2] + i];
    const cd pre = times_i(cd{0.25 * g.hs * nd[4], 0.0});  // (i/4) hs speed
    const cd csig = pre * sg;
    const cd pmu = pre * mu;
    // (k/2)(n_x - i n_y) for G_{n-1}, -(k/2)(n_x + i n_y) for G_{n+1}
    const cd cmuA = cd{0.5 * k * nd[2], -0.5 * k * nd[3]} * pmu;
    const cd cmuB = cd{-0.5 * k * nd[2], -0.5 * k * nd[3]} * pmu;
    cd hp[3], hc[3], ec[3], ep[3];
    double rz2[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double vx = sx0 + (l - 1) * g.d - xj, vy = syp - yj;
      const double r = sqrt(vx * vx + vy * vy);
      const double z = k * r;
      const double ir = 1.0 / r;
      ec[l] = cd{vx * ir, -vy * ir};  // e^{-i theta}
      ep[l] = ec[l];
      rz2[l] = 2.0 / z;
      cd h0, h1;
      hankel01_tab(z, stab, h0, h1);
      hp[l] = wl[l] * h0;
      hc[l] = wl[l] * h1;
      // one copy after another: keeps the table reads of the copies from being
      // scheduled together (register peak)
      asm volatile("" ::: "memory");
    }
    // order 0: G_0 -> acc[0] (sigma), acc[+1] (as G_{n-1}) and acc[-1] (as G_{n+1})
    const cd G0 = hp[0] + hp[1] + hp[2];
    cmac(acc[P], csig, G0);
    if (P >= 1) {
      cmac(acc[P + 1], cmuA, G0);
      cmac(acc[P - 1], cmuB, G0);
    }
#pragma unroll
    for (int m = 1; m <= P + 1; ++m) {
      // G_m = sum H_m e^{-im theta}, G_{-m} = (-1)^m sum H_m e^{im theta}
      cd Gp{0, 0}, Gm{0, 0};
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        Gp.r = fma(hc[l].r, ep[l].r, Gp.r);
        Gp.r = fma(-hc[l].i, ep[l].i, Gp.r);
        Gp.i = fma(hc[l].r, ep[l].i, Gp.i);
        Gp.i = fma(hc[l].i, ep[l].r, Gp.i);
        Gm.r = fma(hc[l].r, ep[l].r, Gm.r);
        Gm.r = fma(hc[l].i, ep[l].i, Gm.r);
        Gm.i = fma(hc[l].i, ep[l].r, Gm.i);
        Gm.i = fma(-hc[l].r, ep[l].i, Gm.i);
      }
      if (m & 1) Gm = -Gm;
      if (m <= P) {
        cmac(acc[P + m], csig, Gp);
        cmac(acc[P - m], csig, Gm);
      }
      // G_m feeds acc[m - 1] (as G_{n+1}) and acc[m + 1] (as G_{n-1}); G_{-m} feeds
      // acc[-m + 1] (as G_{n-1}) and acc[-m - 1] (as G_{n+1})
      if (m - 1 <= P) cmac(acc[P + m - 1], cmuB, Gp);
      if (m + 1 <= P) cmac(acc[P + m + 1], cmuA, Gp);
      if (1 - m >= -P) cmac(acc[P + 1 - m], cmuA, Gm);
      if (-m - 1 >= -P) cmac(acc[P - m - 1], cmuB, Gm);
      if (m <= P) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const cd hn = (m * rz2[l]) * hc[l] - hp[l];
          hp[l] = hc[l];
          hc[l] = hn;
          ep[l] = ep[l] * ec[l];
        }
      }
    }
  }
  // the waves' sums through LDS: wave 3, then 2, then 1 add into the buffer in
  // turn, wave 0 adds its own and stores
  for (int src = BX_WAVES - 1; src >= 1; --src) {
    __syncthreads();
    if (wv == src) {
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        cd v = acc[n];
        if (src != BX_WAVES - 1) v += red[n * 64 + lane];
        red[n * 64 + lane] = v;
      }
    }
  }
  __syncthreads();
  if (wv == 0 && live) {
    cd* out = partial + ((size_t)by_ * g.M + j) * NB;
#pragma unroll
    for (int n = 0; n < NB; ++n) out[n] = acc[n] + red[n * 64 + lane];
  }
}

// L2L of the middle-layer J expansion (coefficients a2, orders -Q2..Q2) to the
// incoming coefficients of ntb (at most L2L_TARGETS) targets per 256-thread block:
//   out[j][n] = sum_q a2_q E_j[q - n],  E_j[m] = J_m(k2 rho_j) e^{i m phi_j},
// E_j stored at offset L = Q2 + P.  a2 and the block's E rows are staged in LDS
// (extern shared: 2 Q2 + 1 + ntb (2L + 1) complex, see l2l_targets_per_block); one
// thread per (target, n), consecutive n reading consecutive LDS entries.
constexpr int L2L_TARGETS = 2;   // few targets per block: many blocks for M ~ 1000
constexpr size_t L2L_LDS_BUDGET = 60 * 1024;
// targets per block so that the staged rows fit the LDS budget
__host__ __device__ inline int l2l_targets_per_block(int P, int Q2) {
  const size_t row = sizeof(cd) * (size_t)(2 * (Q2 + P) + 1);
  const size_t fixed = sizeof(cd) * (size_t)(2 * Q2 + 1);
  int n = fixed + row <= L2L_LDS_BUDGET ? (int)((L2L_LDS_BUDGET - fixed) / row) : 1;
  return n < 1 ? 1 : (n > L2L_TARGETS ? L2L_TARGETS : n);
}
__host__ __device__ inline size_t l2l_lds_bytes(int P, int Q2, int ntb) {
  return sizeof(cd) * (size_t)(2 * Q2 + 1 + ntb * (2 * (Q2 + P) + 1));
}
__device__ inline void l2l_block(int M, int P, int Q2, const cd* __restrict__ E,
                                 const cd* __restrict__ a2, cd* out, int bx_, int ntb) {
  extern __shared__ cd l2l_smem[];
  const int NB = 2 * P + 1;
  const int L = Q2 + P;
  const int row = 2 * L + 1;
  cd* sa = l2l_smem;
  cd* se = l2l_smem + 2 * Q2 + 1;
  const int j0 = bx_ * ntb;
  const int nt = min(ntb, M - j0);
  for (int i = threadIdx.x; i < 2 * Q2 + 1; i += blockDim.x) sa[i] = a2[i];
  for (int i = threadIdx.x; i < nt * row; i += blockDim.x) se[i] = E[(size_t)j0 * row + i];
  __syncthreads();
  for (int t = threadIdx.x; t < nt * NB; t += blockDim.x) {
    const int jj = t / NB, nn = t - jj * NB;
    const cd* e = se + jj * row + L - (nn - P);
    cd acc{0, 0};
    for (int q = -Q2; q <= Q2; ++q) cmac(acc, sa[q + Q2], e[q]);
    out[(size_t)(j0 + jj) * NB + nn] = acc;
  }
}


}  // namespace grt
