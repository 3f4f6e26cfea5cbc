// Translation of many right-hand sides at once on FP32 matrix cores (paper sec. 4.2,
// eq. trans / scattmatrix with the Bloch phase of eq. repre3_mod).
//
// R incidence angles on one geometry share everything in the translation but the
// Bloch phase alpha_r = e^{i kappa_r d} of the near copies l = -1, 0, 1: for target j
//
//   (S T_r x_r)_j[n] = s_j[n] sum_{m, l} alpha_r^l sum_nu H_{nu-n}(k2 rho_l) e^{i(nu-n) phi_l} x_r,m[nu],
//   rho_l e^{i phi_l} = c_j - c_m - l d e_x,   (j, m, l) != (j, j, 0).
//
// In the basis normalised by D = |H_|n|(k2 r)| (x^ = D x) every entry of
// D S T D^{-1} is at most of order one (the multipole series of two disjoint disks
// converges), so the product runs in FP32 without range trouble:
//
//   Y[(j, n), r] = sum_{(m, l, nu)} A_j[n, (m, l, nu)] B[(m, l, nu), r],
//   A_j[n, (m, l, nu)] = D_j[n] s_j[n] tau^{(jml)}_{nu-n} / D_m[nu]   (generated, FP64 -> FP32)
//   B[(m, l, nu), r]   = alpha_r^l x^_r,m[nu]                        (FP32, phase in registers)
//
// a complex GEMM with K = 3 M (2P+1): four real v_mfma_f32_16x16x4f32 per complex
// step.  Work-group: four waves, one target each (its 2P+1 rows padded to 48 = three
// 16-row tiles), sharing 64 right-hand sides (four 16-column tiles).  The generator
// tau of each (target, source, copy) is computed in FP64 by the Hankel recurrence
// (four sources per round, one lane each per copy) into the wave's own LDS; the B
// fragments are read from global memory (the same 64 columns for all four waves, so
// L2 serves three of every four reads).
//
// Layouts: X [M][NBK][Rp] and Y [M][NB][Rp] complex FP32, r fastest (NB = 2P+1,
// NBK = NB rounded up to a multiple of 4 with zero rows, Rp = R rounded up to 64 with
// zero columns); phases [Rp].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BLK_WAVES = 4;   // targets per work-group
constexpr int BLK_COLS = 64;   // right-hand sides per work-group (four 16-column tiles)
constexpr int BLK_SB = 4;      // sources per generator round

template <int P>
struct BlkShape {
  static constexpr int NB = 2 * P + 1;
  static constexpr int NQ = 4 * P + 1;
  static constexpr int NS = (NB + 3) / 4;        // K steps of 4 per (source, copy)
  static constexpr int NBK = 4 * NS;
  static constexpr int MT = (NB + 15) / 16;      // 16-row tiles per target
};

template <int P>
__global__ void __launch_bounds__(64 * BLK_WAVES)
    block_st_kernel(const double* __restrict__ cx, const double* __restrict__ cy, int M,
                    double k2, double d, const double* __restrict__ dnorm,
                    const cd* __restrict__ mie, const double* __restrict__ dinv,
                    const double* __restrict__ htab, const cf* __restrict__ X, int Rp,
                    const cf* __restrict__ phase, cf* __restrict__ Y) {
  using S = BlkShape<P>;
  constexpr int NB = S::NB, NQ = S::NQ, NS = S::NS, NBK = S::NBK, MT = S::MT;
  __shared__ cd tau_s[BLK_WAVES][BLK_SB][3][NQ];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.x * BLK_WAVES + wv;
  const bool live = j < M;
  const int jj = live ? j : M - 1;
  const int col0 = blockIdx.y * BLK_COLS;
  const int li = lane & 15, lk = lane >> 4;   // A row / B column; K index
  const double xj = cx[jj], yj = cy[jj];
  // E_j[n] = D_j[n] s_j[n] for this lane's row in each 16-row tile
  cd E[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int n = mt * 16 + li;
    E[mt] = n < NB ? dnorm[(size_t)jj * NB + n] * mie[(size_t)jj * NB + n] : cd{0.0, 0.0};
  }
  // alpha_r of this lane's column in each 16-column tile
  cf ph[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) ph[nt] = phase[col0 + nt * 16 + li];
  v4f accr[MT][4], acci[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      accr[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
      acci[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  for (int m0 = 0; m0 < M; m0 += BLK_SB) {
    const int nsb = min(BLK_SB, M - m0);
    __syncthreads();   // the previous round's generators are no longer read
    if (lane < 3 * BLK_SB) {
      const int sb = lane / 3, l = lane % 3 - 1;
      cd* t = tau_s[wv][sb][l + 1];
      const int m = m0 + sb;
      if (sb >= nsb || (m == jj && l == 0)) {
        for (int q = 0; q < NQ; ++q) t[q] = cd{0.0, 0.0};
      } else {
        const double dx = xj - cx[m] - l * d, dy = yj - cy[m];
        const double rho = sqrt(dx * dx + dy * dy);
        const double z = k2 * rho;
        const cd e{dx / rho, dy / rho};
        cd hm, hc;   // H_{q-1}, H_q
        hankel01_tab(z, htab, hm, hc);
        t[2 * P] = hm;   // q = 0
        cd ep = e;       // e^{i q phi}
        const double i2z = 2.0 / z;
        for (int q = 1; q <= 2 * P; ++q) {
          // hc = H_q
          const cd v = hc * ep;
          t[2 * P + q] = v;
          const cd w = hc * conj(ep);
          t[2 * P - q] = (q & 1) ? -w : w;   // H_{-q} e^{-iq phi} = (-1)^q H_q e^{-iq phi}
          const cd hn = (q * i2z) * hc - hm;
          hm = hc;
          hc = hn;
          ep = ep * e;
        }
      }
    }
    __syncthreads();
    for (int sb = 0; sb < nsb; ++sb) {
      const int m = m0 + sb;
      const cf* xm = X + (size_t)m * NBK * Rp + col0 + li;
      const double* dim = dinv + (size_t)m * NB;
      for (int s = 0; s < NS; ++s) {
        const int kv = 4 * s + lk;   // nu index of this lane's K slot
        cf xb[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) xb[nt] = xm[(size_t)kv * Rp + nt * 16];
        const double dv = kv < NB ? dim[kv] : 0.0;
#pragma unroll
        for (int l = -1; l <= 1; ++l) {
          const cd* t = tau_s[wv][sb][l + 1];
          float ar[MT], ai[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int n = mt * 16 + li;
            cd a{0.0, 0.0};
            if (n < NB && kv < NB) a = (dv * E[mt]) * t[2 * P + kv - n];
            ar[mt] = (float)a.r;
            ai[mt] = (float)a.i;
          }
          float br[4], bi[4];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            if (l == 0) {
              br[nt] = xb[nt].r;
              bi[nt] = xb[nt].i;
            } else {
              // alpha^l x, alpha^{-1} = conj(alpha)
              const float pr = ph[nt].r, pi = l > 0 ? ph[nt].i : -ph[nt].i;
              br[nt] = pr * xb[nt].r - pi * xb[nt].i;
              bi[nt] = pr * xb[nt].i + pi * xb[nt].r;
            }
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
              accr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], br[nt], accr[mt][nt], 0, 0, 0);
              acci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], bi[nt], acci[mt][nt], 0, 0, 0);
            }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
              accr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[mt], bi[nt], accr[mt][nt], 0, 0, 0);
              acci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mt], br[nt], acci[mt][nt], 0, 0, 0);
            }
        }
      }
    }
  }
  if (!live) return;
  // lane holds rows 4 (lane / 16) + v of each 16-row tile, column lane % 16
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = mt * 16 + 4 * lk + v;
      if (n >= NB) continue;
      cf* yr = Y + ((size_t)j * NB + n) * Rp + col0 + li;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) yr[nt * 16] = cf{accr[mt][nt][v], acci[mt][nt][v]};
    }
}

// X[m][k][r] = D x_r[m][k] (FP32) for k < NB, zero for the padding rows and columns.
__global__ void block_pack_kernel(const cd* __restrict__ x, int64_t ldx, const double* dn,
                                  int M, int NB, int NBK, int R, int Rp, cf* X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)M * NBK * Rp;
  if (i >= tot) return;
  const int r = (int)(i % Rp);
  const int64_t mk = i / Rp;
  const int k = (int)(mk % NBK);
  const int m = (int)(mk / NBK);
  cf v{0.f, 0.f};
  if (r < R && k < NB) {
    const int64_t e = (int64_t)m * NB + k;
    const cd xv = x[(size_t)r * ldx + e];
    const double s = dn ? dn[e] : 1.0;
    v = cf{(float)(s * xv.r), (float)(s * xv.i)};
  }
  X[i] = v;
}

// y_r = x_r - D^{-1} Y_r + s o w_r  (w_r = B_phys A^+ C x_r): the mixed K x_r with the
// block translation, in the unnormalised basis, FP64 out.
__global__ void block_combine_kernel(const cd* __restrict__ x, const cf* __restrict__ Yb,
                                     const cd* __restrict__ w, const double* __restrict__ dinv,
                                     const cd* __restrict__ mie, int64_t nbeta, int R, int Rp,
                                     cd* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbeta * R) return;
  const int r = (int)(i / nbeta);
  const int64_t e = i - (int64_t)r * nbeta;
  const cf t = Yb[(size_t)e * Rp + r];
  y[i] = x[i] - dinv[e] * cd{t.r, t.i} + mie[e] * w[i];
}

// y_r = D^{-1} Y_r: S T x_r from the block product (diagnostics).
__global__ void block_unpack_kernel(const cf* __restrict__ Yb, const double* __restrict__ dinv,
                                    int64_t nbeta, int R, int Rp, cd* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbeta * R) return;
  const int r = (int)(i / nbeta);
  const int64_t e = i - (int64_t)r * nbeta;
  const cf t = Yb[(size_t)e * Rp + r];
  y[i] = dinv[e] * cd{t.r, t.i};
}

template <int P>
void launch_block(grt_ctx* c, hipStream_t s) {
  dim3 grid((unsigned)((c->M + BLK_WAVES - 1) / BLK_WAVES), (unsigned)(c->blk_Rp / BLK_COLS));
  block_st_kernel<P><<<grid, 64 * BLK_WAVES, 0, s>>>(
      c->d_cx, c->d_cy, (int)c->M, c->g.k[1], c->g.d, c->d_dnorm, c->d_mie, c->d_dinv,
      c->d_htab, c->d_blkX, c->blk_Rp, c->d_blkph, c->d_blkY);
}

}  // namespace

int block_nbk(int P) { return 4 * ((2 * P + 1 + 3) / 4); }

// Buffers of the block product for R right-hand sides (phases from the contexts of
// the angles, alpha_r = e^{i kappa_r d}).
grt_status block_prepare(grt_ctx* c, int R, const cd* alphas_host) {
  const int Rp = ((R + BLK_COLS - 1) / BLK_COLS) * BLK_COLS;
  if (Rp != c->blk_Rp || !c->d_blkX) {
    if (c->d_blkX) hipFree(c->d_blkX);
    if (c->d_blkY) hipFree(c->d_blkY);
    if (c->d_blkph) hipFree(c->d_blkph);
    c->d_blkX = c->d_blkY = nullptr;
    c->d_blkph = nullptr;
    c->blk_Rp = 0;
    const size_t nx = (size_t)c->M * block_nbk(c->P) * Rp, ny = (size_t)c->n_beta * Rp;
    GRT_HIP(c, hipMalloc(&c->d_blkX, sizeof(cf) * nx));
    GRT_HIP(c, hipMalloc(&c->d_blkY, sizeof(cf) * ny));
    GRT_HIP(c, hipMalloc(&c->d_blkph, sizeof(cf) * Rp));
    c->blk_Rp = Rp;
  }
  std::vector<cf> ph(Rp, cf{1.f, 0.f});
  for (int r = 0; r < R; ++r) ph[r] = cf{(float)alphas_host[r].r, (float)alphas_host[r].i};
  GRT_HIP(c, hipMemcpyAsync(c->d_blkph, ph.data(), sizeof(cf) * Rp, hipMemcpyHostToDevice,
                            c->stream));
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  return GRT_OK;
}

// Y = D S T D^{-1} X for every column: X packed from R vectors x (stride ldx), scaled
// by D when dn is given (x unnormalised) or taken as is (x already normalised).
grt_status block_product(grt_ctx* c, const cd* x, int64_t ldx, const double* dn, int R,
                         hipStream_t s) {
  const int NB = c->nb, NBK = block_nbk(c->P);
  const int64_t tot = (int64_t)c->M * NBK * c->blk_Rp;
  block_pack_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(x, ldx, dn, (int)c->M, NB, NBK,
                                                                   R, c->blk_Rp, c->d_blkX);
  switch (c->P) {
    case 1: launch_block<1>(c, s); break;
    case 2: launch_block<2>(c, s); break;
    case 3: launch_block<3>(c, s); break;
    case 4: launch_block<4>(c, s); break;
    case 5: launch_block<5>(c, s); break;
    case 6: launch_block<6>(c, s); break;
    case 8: launch_block<8>(c, s); break;
    case 10: launch_block<10>(c, s); break;
    case 12: launch_block<12>(c, s); break;
    case 15: launch_block<15>(c, s); break;
    case 20: launch_block<20>(c, s); break;
    default: return set_err(c, GRT_EUNSUP, "multipole order P not compiled in");
  }
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

void block_combine(grt_ctx* c, const cd* x, const cd* w, int R, cd* y, hipStream_t s) {
  const int64_t n = c->n_beta * R;
  block_combine_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
      x, c->d_blkY, w, c->d_dinv, c->d_mie, c->n_beta, R, c->blk_Rp, y);
}

void block_unpack(grt_ctx* c, int R, cd* y, hipStream_t s) {
  const int64_t n = c->n_beta * R;
  block_unpack_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c->d_blkY, c->d_dinv,
                                                                  c->n_beta, R, c->blk_Rp, y);
}
