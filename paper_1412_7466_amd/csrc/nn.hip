// Learned warm start for the GMRES solve: a message-passing network over each
// inclusion's K nearest neighbours (minimum image in x) predicts the multiple-
// scattering correction of the incoming coefficients on orders |n| <= p_out, and
// the initial guess is beta0 = s (alpha0 + correction), alpha0 = B_phys A^+ f the
// incoming coefficients of the layers alone (sec. 5), s the Mie diagonal (sec. 4.1).
//
// Network (width H, L layers, F = 32 node inputs, E = 8 edge inputs, O = 2(2 p_out+1)
// outputs; weights in bfloat16, activations and accumulation in FP32, every GEMM on
// the FP32 matrix cores):
//   h0 = relu(W_in f + b_in)
//   per layer: P = A h, Q = B h;  msg_jk = relu(P_j + Q_nbr(j,k) + C e_jk + c)
//              agg_j = mean_k msg_jk;  h <- h + relu(U [h; agg] + u)
//   out = W_out h + b_out
// Training minimises sum w |out - t|^2 / wnorm per geometry with Adam (FP32 master
// weights, bfloat16 copy used by the forward and backward passes).  Every pass is a
// chain of the kernels below; the message backward is deterministic (no atomics:
// the scatter to neighbours runs over a reverse adjacency list).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

constexpr int NF = 32;    // node inputs
constexpr int NE = 8;     // edge inputs
constexpr int KMAX = 32;  // most neighbours per node

__device__ __forceinline__ float ld_val(float v) { return v; }
__device__ __forceinline__ float ld_val(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// round to nearest bfloat16, ties to even
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

enum { EPI_PLAIN = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_BIAS_RESID = 3 };

typedef float v4f __attribute__((ext_vector_type(4)));

// C[i][j] = alpha sum_k A(i,k) B(k,j) + beta C[i][j], A(i,k) = A[i sai + k sak],
// B(k,j) = B[k sbk + j sbn], on the matrix cores: one wave per 16x16 output tile,
// v_mfma_f32_16x16x4f32 over K in steps of 4 (lane l holds A(i0 + l % 16, k0 + l / 16)
// and B(k0 + l / 16, j0 + l % 16); the accumulator rows 4 (l / 16) + v, column l % 16).
// B in bfloat16 (the weights) is widened to FP32 exactly, so the products and the
// FP32 accumulation see the rounded weights and full FP32 activations.  Epilogues:
// EPI_BIAS C = AB + bias[j]; EPI_BIAS_RELU also D = relu(C); EPI_BIAS_RESID also
// D = R + relu(C).
template <typename TBv, int EPI>
__global__ void __launch_bounds__(64) gemm_kernel(int Mr, int Nc, int Kd, const float* __restrict__ A,
                                                  int64_t sai, int64_t sak, const TBv* __restrict__ B,
                                                  int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                                                  float alpha, float beta, const TBv* __restrict__ bias,
                                                  float* D, int64_t ldd, const float* R, int64_t ldr) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int ai = i0 + li, bj = j0 + li;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Kd; k0 += 4) {
    const int k = k0 + lk;
    const float a = (ai < Mr && k < Kd) ? A[ai * sai + k * sak] : 0.f;
    const float b = (k < Kd && bj < Nc) ? ld_val(B[k * sbk + bj * sbn]) : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  const int j = j0 + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 4 * lk + v;
    if (i >= Mr || j >= Nc) continue;
    if (EPI == EPI_PLAIN) {
      float w = alpha * acc[v];
      if (beta != 0.f) w += beta * C[i * ldc + j];
      C[i * ldc + j] = w;
    } else {
      const float pre = acc[v] + ld_val(bias[j]);
      C[i * ldc + j] = pre;
      if (EPI == EPI_BIAS_RELU) D[i * ldd + j] = fmaxf(pre, 0.f);
      if (EPI == EPI_BIAS_RESID) D[i * ldd + j] = R[i * ldr + j] + fmaxf(pre, 0.f);
    }
  }
}

// out[c] = sum over rows of in[r * ld + c] (fixed order)
__global__ void colsum_kernel(int rows, int cols, const float* in, int64_t ld, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += in[r * ld + c];
  out[c] = s;
}

// y[i][c] = x[i][c] * (mask[i][c] > 0)   (all [rows][cols], leading dims given)
__global__ void relu_mask_kernel(int rows, int cols, const float* x, int64_t ldx, const float* mask,
                                 int64_t ldm, float* y, int64_t ldy) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int64_t i = t / cols, c = t - i * cols;
  y[i * ldy + c] = mask[i * ldm + c] > 0.f ? x[i * ldx + c] : 0.f;
}

// y[i][c] += x[i][c]
__global__ void add_kernel(int rows, int cols, const float* x, int64_t ldx, float* y, int64_t ldy) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int64_t i = t / cols, c = t - i * cols;
  y[i * ldy + c] += x[i * ldx + c];
}

// Message forward of one layer: one block per node j, one thread per channel c.
// agg[j][c] = mean over valid k of relu(P[j][c] + c_b[c] + Q[m][c] + sum_e C[c][e] e_jk[e]),
// written to Z[j][H + c].
__global__ void edge_fwd_kernel(int H, int K, const int* __restrict__ nbr, const int* __restrict__ cnt,
                                const float* __restrict__ edge, const float* __restrict__ P,
                                const float* __restrict__ Q, const uint16_t* __restrict__ Cw,
                                const uint16_t* __restrict__ cb, float* Z, int64_t ldz) {
  __shared__ float es[KMAX * NE];
  __shared__ int ns[KMAX];
  const int j = blockIdx.x, c = threadIdx.x;
  for (int t = c; t < K * NE; t += blockDim.x) es[t] = edge[(int64_t)j * K * NE + t];
  for (int t = c; t < K; t += blockDim.x) ns[t] = nbr[(int64_t)j * K + t];
  __syncthreads();
  if (c >= H) return;
  float w[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) w[e] = ld_val(Cw[c * NE + e]);
  const float base = P[(int64_t)j * H + c] + ld_val(cb[c]);
  float sum = 0.f;
  for (int k = 0; k < K; ++k) {
    const int m = ns[k];
    if (m < 0) continue;
    float pre = base + Q[(int64_t)m * H + c];
#pragma unroll
    for (int e = 0; e < NE; ++e) pre = fmaf(w[e], es[k * NE + e], pre);
    sum += fmaxf(pre, 0.f);
  }
  const int n = cnt[j];
  Z[(int64_t)j * ldz + H + c] = n > 0 ? sum / (float)n : 0.f;
}

// Message backward, target side: dP[j][c] = sum_k dm_jkc and per-node partials
// part[j][c][e] = sum_k dm_jkc e_jk[e], part[j][c][NE] = sum_k dm_jkc, with
// dm_jkc = dagg[j][c] / cnt_j * [pre_jkc > 0] (pre recomputed as in the forward).
__global__ void edge_bwd_kernel(int H, int K, const int* __restrict__ nbr, const int* __restrict__ cnt,
                                const float* __restrict__ edge, const float* __restrict__ P,
                                const float* __restrict__ Q, const uint16_t* __restrict__ Cw,
                                const uint16_t* __restrict__ cb, const float* __restrict__ dZ,
                                int64_t ldz, float* dP, float* part) {
  __shared__ float es[KMAX * NE];
  __shared__ int ns[KMAX];
  const int j = blockIdx.x, c = threadIdx.x;
  for (int t = c; t < K * NE; t += blockDim.x) es[t] = edge[(int64_t)j * K * NE + t];
  for (int t = c; t < K; t += blockDim.x) ns[t] = nbr[(int64_t)j * K + t];
  __syncthreads();
  if (c >= H) return;
  float w[NE], acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    w[e] = ld_val(Cw[c * NE + e]);
    acc[e] = 0.f;
  }
  const int n = cnt[j];
  const float g = n > 0 ? dZ[(int64_t)j * ldz + H + c] / (float)n : 0.f;
  const float base = P[(int64_t)j * H + c] + ld_val(cb[c]);
  float sp = 0.f;
  for (int k = 0; k < K; ++k) {
    const int m = ns[k];
    if (m < 0) continue;
    float pre = base + Q[(int64_t)m * H + c];
#pragma unroll
    for (int e = 0; e < NE; ++e) pre = fmaf(w[e], es[k * NE + e], pre);
    if (pre > 0.f) {
      sp += g;
#pragma unroll
      for (int e = 0; e < NE; ++e) acc[e] = fmaf(g, es[k * NE + e], acc[e]);
    }
  }
  dP[(int64_t)j * H + c] = sp;
  float* pp = part + ((int64_t)j * H + c) * (NE + 1);
#pragma unroll
  for (int e = 0; e < NE; ++e) pp[e] = acc[e];
  pp[NE] = sp;
}

// Message backward, source side: dQ[m][c] = sum over edges (j, k) with nbr = m of
// dm_jkc, over the reverse adjacency list of m (entries j * K + k, ascending).
__global__ void edge_bwd_q_kernel(int H, int K, const int* __restrict__ rev_off,
                                  const int* __restrict__ rev, const int* __restrict__ cnt,
                                  const float* __restrict__ edge, const float* __restrict__ P,
                                  const float* __restrict__ Q, const uint16_t* __restrict__ Cw,
                                  const uint16_t* __restrict__ cb, const float* __restrict__ dZ,
                                  int64_t ldz, float* dQ) {
  const int m = blockIdx.x, c = threadIdx.x;
  if (c >= H) return;
  float w[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) w[e] = ld_val(Cw[c * NE + e]);
  const float cbc = ld_val(cb[c]);
  const float qm = Q[(int64_t)m * H + c];
  float s = 0.f;
  for (int r = rev_off[m]; r < rev_off[m + 1]; ++r) {
    const int jk = rev[r];
    const int j = jk / K;
    float pre = P[(int64_t)j * H + c] + cbc;
    pre = pre + qm;
    const float* ee = edge + (int64_t)jk * NE;
#pragma unroll
    for (int e = 0; e < NE; ++e) pre = fmaf(w[e], ee[e], pre);
    if (pre > 0.f) s += dZ[(int64_t)j * ldz + H + c] / (float)cnt[j];
  }
  dQ[(int64_t)m * H + c] = s;
}

// Scatter the reduced message partials [H][NE+1] into the C and c gradient slots.
__global__ void split_partials_kernel(int H, const float* red, float* gC, float* gc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= H) return;
  for (int e = 0; e < NE; ++e) gC[c * NE + e] = red[c * (NE + 1) + e];
  gc[c] = red[c * (NE + 1) + NE];
}

// Weighted squared error: dout = 2 w (out - t) / wnorm; per-block partial sums of
// w (out - t)^2 (FP64) for a fixed-order total.
__global__ void __launch_bounds__(256) loss_kernel(int64_t n, const float* out, const float* t,
                                                   const float* w, double inv_wnorm, float* dout,
                                                   double* part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const float dlt = out[i] - t[i];
    v = (double)w[i] * (double)dlt * (double)dlt;
    dout[i] = (float)(2.0 * (double)w[i] * (double)dlt * inv_wnorm);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_finish_kernel(int nb, const double* part, double inv_wnorm, double* dst) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *dst = s * inv_wnorm;
}

__global__ void adam_kernel(int64_t n, float* p, const float* g, float* m1, float* m2, uint16_t* pb,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  p[i] = v;
  pb[i] = to_bf16(v);
}

__global__ void round_bf16_kernel(int64_t n, const float* p, uint16_t* pb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = to_bf16(p[i]);
}

// ---------------------------------------------------------------------------
// graph and features
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wrap_dx(double dx, double d) {
  if (dx > 0.5 * d) dx -= d;
  else if (dx < -0.5 * d) dx += d;
  return dx;
}

// K nearest other inclusions of j (minimum image in x), ascending distance, ties
// by index; -1 beyond the M-1 others.  One thread per target.
__global__ void knn_kernel(int M, int K, const double* __restrict__ x, const double* __restrict__ y,
                           double d, int* nbr, int* cnt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double bd[KMAX];
  int bi[KMAX];
  int n = 0;
  const double xj = x[j], yj = y[j];
  for (int m = 0; m < M; ++m) {
    if (m == j) continue;
    const double dx = wrap_dx(xj - x[m], d);
    const double dy = yj - y[m];
    const double r2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
    if (n == K && !(r2 < bd[K - 1])) continue;
    int p = n < K ? n : K - 1;
    while (p > 0 && r2 < bd[p - 1]) {
      bd[p] = bd[p - 1];
      bi[p] = bi[p - 1];
      --p;
    }
    bd[p] = r2;
    bi[p] = m;
    if (n < K) ++n;
  }
  for (int k = 0; k < K; ++k) nbr[(int64_t)j * K + k] = k < n ? bi[k] : -1;
  cnt[j] = n;
}

// e_jk = [k dx, k dy, z, 1/z, H0(z), H1(z) e^{i phi}] with z = k rho, rho e^{i phi} = c_j - c_m.
__global__ void edge_feat_kernel(int M, int K, const int* __restrict__ nbr, const double* __restrict__ x,
                                 const double* __restrict__ y, double d, double k2, float* edge) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * K) return;
  const int j = (int)(t / K);
  const int m = nbr[t];
  float* e = edge + t * NE;
  if (m < 0) {
    for (int i = 0; i < NE; ++i) e[i] = 0.f;
    return;
  }
  const double dx = wrap_dx(x[j] - x[m], d);
  const double dy = y[j] - y[m];
  const double rho = sqrt(dx * dx + dy * dy);
  const double z = k2 * rho;
  cd h0, h1;
  hankel01(z, h0, h1);
  const cd eph{dx / rho, dy / rho};
  const cd h1e = h1 * eph;
  e[0] = (float)(k2 * dx);
  e[1] = (float)(k2 * dy);
  e[2] = (float)z;
  e[3] = (float)(1.0 / z);
  e[4] = (float)h0.r;
  e[5] = (float)h0.i;
  e[6] = (float)h1e.r;
  e[7] = (float)h1e.i;
}

// Node inputs: k2 r, n/n2 - 1, y/h, sin phi, omega/40, D s for n = 0, 1, 2 and alpha0
// for n = -3..3 (re, im), zero padding to NF.
__global__ void node_feat_kernel(int M, int P, double k2, double h, double sinphi, double omega,
                                 const double* __restrict__ rad, const double* __restrict__ kp,
                                 const double* __restrict__ y, const double* __restrict__ dn,
                                 const cd* __restrict__ s, const cd* __restrict__ a0, float* feat) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int nb = 2 * P + 1;
  float* f = feat + (int64_t)j * NF;
  for (int i = 0; i < NF; ++i) f[i] = 0.f;
  f[0] = (float)(k2 * rad[j]);
  f[1] = (float)(kp[j] / k2 - 1.0);
  f[2] = (float)(y[j] / h);
  f[3] = (float)sinphi;
  f[4] = (float)(omega / 40.0);
  for (int n = 0; n < 3; ++n) {
    if (n > P) break;
    const int64_t q = (int64_t)j * nb + P + n;
    f[5 + 2 * n] = (float)(dn[q] * s[q].r);
    f[6 + 2 * n] = (float)(dn[q] * s[q].i);
  }
  for (int n = -3; n <= 3; ++n) {
    if (n < -P || n > P) continue;
    const cd v = a0[(int64_t)j * nb + P + n];
    f[11 + 2 * (n + 3)] = (float)v.r;
    f[12 + 2 * (n + 3)] = (float)v.i;
  }
}

// Training target from a solution: t = (T beta - B_phys A^+ C beta) on |n| <= p_out,
// w = (D |s|)^2, and per-node sums of w |alpha0 + correction|^2.
__global__ void target_kernel(int M, int P, int p_out, const cd* __restrict__ Tb,
                              const cd* __restrict__ Lb, const cd* __restrict__ a0,
                              const cd* __restrict__ s, const double* __restrict__ dn, float* t,
                              float* w, double* wpart) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int nb = 2 * P + 1, O = 2 * (2 * p_out + 1);
  double acc = 0.0;
  for (int n = -p_out; n <= p_out; ++n) {
    const int o = 2 * (n + p_out);
    if (n < -P || n > P) {
      t[(int64_t)j * O + o] = t[(int64_t)j * O + o + 1] = 0.f;
      w[(int64_t)j * O + o] = w[(int64_t)j * O + o + 1] = 0.f;
      continue;
    }
    const int64_t q = (int64_t)j * nb + P + n;
    const cd cr = Tb[q] - Lb[q];
    const double ww = dn[q] * dn[q] * cabs2(s[q]);
    t[(int64_t)j * O + o] = (float)cr.r;
    t[(int64_t)j * O + o + 1] = (float)cr.i;
    w[(int64_t)j * O + o] = (float)ww;
    w[(int64_t)j * O + o + 1] = (float)ww;
    acc += ww * cabs2(a0[q] + cr);
  }
  wpart[j] = acc;
}

// beta0[j][n] = s (alpha0 + out) for |n| <= p_out, s alpha0 otherwise.
__global__ void warm_kernel(int M, int P, int p_out, const cd* __restrict__ s, const cd* __restrict__ a0,
                            const float* __restrict__ out, cd* beta0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = 2 * P + 1;
  if (t >= (int64_t)M * nb) return;
  const int j = (int)(t / nb), n = (int)(t - (int64_t)j * nb) - P;
  cd a = a0[t];
  if (n >= -p_out && n <= p_out) {
    const int O = 2 * (2 * p_out + 1), o = 2 * (n + p_out);
    a.r += out[(int64_t)j * O + o];
    a.i += out[(int64_t)j * O + o + 1];
  }
  beta0[t] = s[t] * a;
}

struct Sample {
  int M = 0;
  float *feat = nullptr, *edge = nullptr, *tgt = nullptr, *w = nullptr;
  int *nbr = nullptr, *cnt = nullptr, *rev_off = nullptr, *rev = nullptr;
  double wnorm = 0.0;
  bool has_target = false;
  void release() {
    void* p[] = {feat, edge, tgt, w, nbr, cnt, rev_off, rev};
    for (void* q : p)
      if (q) hipFree(q);
    *this = Sample{};
  }
};

}  // namespace

struct grt_nn {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int H = 128, L = 3, K = 16, p_out = 3, O = 14;
  int64_t np = 0;
  std::vector<int64_t> off;   // offset of every weight tensor in the flat vector
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t* pb = nullptr;
  int64_t t_adam = 0;
  std::vector<Sample> samples;
  // activation workspace, sized for `cap` nodes
  int cap = 0;
  float *pre0 = nullptr, *Z = nullptr, *hL = nullptr, *Pb = nullptr, *Qb = nullptr,
        *upre = nullptr, *out = nullptr, *dout = nullptr, *dh = nullptr, *dz = nullptr,
        *dP = nullptr, *dQ = nullptr, *dtmp = nullptr, *part = nullptr, *red = nullptr;
  double* lpart = nullptr;
  double* losses = nullptr;
  int losses_cap = 0;
};

namespace {

grt_status nset(grt_nn* n, grt_status s, const std::string& m) {
  if (n) n->err = m;
  return s;
}
#define NNHIP(n, call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return nset(n, GRT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)
#define NNTRY(x)                 \
  do {                           \
    grt_status s_ = (x);         \
    if (s_ != GRT_OK) return s_; \
  } while (0)

// tensor indices in the flat layout
inline int T_WIN() { return 0; }
inline int T_BIN() { return 1; }
inline int T_A(int l) { return 2 + 6 * l; }
inline int T_B(int l) { return 3 + 6 * l; }
inline int T_C(int l) { return 4 + 6 * l; }
inline int T_c(int l) { return 5 + 6 * l; }
inline int T_U(int l) { return 6 + 6 * l; }
inline int T_u(int l) { return 7 + 6 * l; }
inline int T_WOUT(int L) { return 2 + 6 * L; }
inline int T_BOUT(int L) { return 3 + 6 * L; }

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename TBv, int EPI>
void gemm(hipStream_t s, int Mr, int Nc, int Kd, const float* A, int64_t sai, int64_t sak,
          const TBv* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc, float alpha = 1.f,
          float beta = 0.f, const TBv* bias = nullptr, float* D = nullptr, int64_t ldd = 0,
          const float* R = nullptr, int64_t ldr = 0) {
  if (Mr <= 0 || Nc <= 0) return;
  dim3 grid(blocks_for(Nc, 16), blocks_for(Mr, 16));
  gemm_kernel<TBv, EPI><<<grid, 64, 0, s>>>(Mr, Nc, Kd, A, sai, sak, B, sbk, sbn, C, ldc, alpha, beta,
                                             bias, D, ldd, R, ldr);
}

grt_status ensure_cap(grt_nn* n, int M) {
  if (M <= n->cap) return GRT_OK;
  float** bufs[] = {&n->pre0, &n->Z, &n->hL, &n->Pb, &n->Qb, &n->upre, &n->out, &n->dout,
                    &n->dh, &n->dz, &n->dP, &n->dQ, &n->dtmp, &n->part, &n->red};
  for (float** b : bufs)
    if (*b) {
      hipFree(*b);
      *b = nullptr;
    }
  if (n->lpart) hipFree(n->lpart);
  n->lpart = nullptr;
  const int cap = std::max(M, 256);
  const size_t H = n->H, L = n->L, O = n->O;
  NNHIP(n, hipMalloc(&n->pre0, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->Z, sizeof(float) * L * cap * 2 * H));
  NNHIP(n, hipMalloc(&n->hL, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->Pb, sizeof(float) * L * cap * H));
  NNHIP(n, hipMalloc(&n->Qb, sizeof(float) * L * cap * H));
  NNHIP(n, hipMalloc(&n->upre, sizeof(float) * L * cap * H));
  NNHIP(n, hipMalloc(&n->out, sizeof(float) * cap * O));
  NNHIP(n, hipMalloc(&n->dout, sizeof(float) * cap * O));
  NNHIP(n, hipMalloc(&n->dh, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->dz, sizeof(float) * cap * 2 * H));
  NNHIP(n, hipMalloc(&n->dP, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->dQ, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->dtmp, sizeof(float) * cap * H));
  NNHIP(n, hipMalloc(&n->part, sizeof(float) * cap * H * (NE + 1)));
  NNHIP(n, hipMalloc(&n->red, sizeof(float) * H * (NE + 1)));
  NNHIP(n, hipMalloc(&n->lpart, sizeof(double) * blocks_for((int64_t)cap * O, 256)));
  n->cap = cap;
  return GRT_OK;
}

// Graph, features and (with beta) the training target of one built context.
grt_status build_sample(grt_nn* n, grt_ctx* c, const cd* beta, Sample* S, cd** a0_out = nullptr) {
  const int M = (int)c->M, P = c->P, K = n->K, O = n->O;
  const int64_t nbeta = c->n_beta;
  hipStream_t s = c->stream;
  *S = Sample{};
  S->M = M;
  cd *a0 = nullptr, *Tb = nullptr, *Lb = nullptr;
  double* wpart = nullptr;
  auto fail = [&](grt_status st) {
    if (a0) hipFree(a0);
    if (Tb) hipFree(Tb);
    if (Lb) hipFree(Lb);
    if (wpart) hipFree(wpart);
    S->release();
    return st;
  };
#define SHIP(call)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(nset(n, GRT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_))); \
  } while (0)
  SHIP(hipMalloc(&a0, sizeof(cd) * nbeta));
  SHIP(hipMalloc(&S->feat, sizeof(float) * (size_t)M * NF));
  SHIP(hipMalloc(&S->edge, sizeof(float) * (size_t)M * K * NE));
  SHIP(hipMalloc(&S->nbr, sizeof(int) * (size_t)M * K));
  SHIP(hipMalloc(&S->cnt, sizeof(int) * (size_t)M));
  grt_status st = incident_alpha(c, a0);
  if (st != GRT_OK) return fail(nset(n, st, "incident field: " + c->err));
  knn_kernel<<<blocks_for(M, 64), 64, 0, s>>>(M, K, c->d_cx, c->d_cy, c->g.d, S->nbr, S->cnt);
  edge_feat_kernel<<<blocks_for((int64_t)M * K, 256), 256, 0, s>>>(M, K, S->nbr, c->d_cx, c->d_cy,
                                                                    c->g.d, c->g.k[1], S->edge);
  node_feat_kernel<<<blocks_for(M, 128), 128, 0, s>>>(M, P, c->g.k[1], c->g.h,
                                                      std::sin(c->inc.phi), c->inc.omega, c->d_rad,
                                                      c->d_kp, c->d_cy, c->d_dnorm, c->d_mie, a0,
                                                      S->feat);
  SHIP(hipGetLastError());
  // reverse adjacency (host: integer bookkeeping only)
  std::vector<int> nb((size_t)M * K);
  SHIP(hipMemcpyAsync(nb.data(), S->nbr, sizeof(int) * nb.size(), hipMemcpyDeviceToHost, s));
  SHIP(hipStreamSynchronize(s));
  std::vector<int> roff(M + 1, 0), rev;
  for (int v : nb)
    if (v >= 0) roff[v + 1]++;
  for (int m = 0; m < M; ++m) roff[m + 1] += roff[m];
  rev.resize(std::max(1, roff[M]));
  {
    std::vector<int> fill(roff.begin(), roff.end() - 1);
    for (int64_t jk = 0; jk < (int64_t)M * K; ++jk)
      if (nb[jk] >= 0) rev[fill[nb[jk]]++] = (int)jk;
  }
  SHIP(hipMalloc(&S->rev_off, sizeof(int) * (M + 1)));
  SHIP(hipMalloc(&S->rev, sizeof(int) * rev.size()));
  SHIP(hipMemcpy(S->rev_off, roff.data(), sizeof(int) * (M + 1), hipMemcpyHostToDevice));
  SHIP(hipMemcpy(S->rev, rev.data(), sizeof(int) * rev.size(), hipMemcpyHostToDevice));
  SHIP(hipMalloc(&S->tgt, sizeof(float) * (size_t)M * O));
  SHIP(hipMalloc(&S->w, sizeof(float) * (size_t)M * O));
  SHIP(hipMemsetAsync(S->tgt, 0, sizeof(float) * (size_t)M * O, s));
  SHIP(hipMemsetAsync(S->w, 0, sizeof(float) * (size_t)M * O, s));
  S->wnorm = 1.0;
  if (beta) {
    SHIP(hipMalloc(&Tb, sizeof(cd) * nbeta));
    SHIP(hipMalloc(&Lb, sizeof(cd) * nbeta));
    SHIP(hipMalloc(&wpart, sizeof(double) * M));
    if ((st = apply_T_only(c, beta, Tb)) != GRT_OK) return fail(nset(n, st, c->err));
    if ((st = apply_lowrank_only(c, beta, Lb)) != GRT_OK) return fail(nset(n, st, c->err));
    target_kernel<<<blocks_for(M, 128), 128, 0, s>>>(M, P, n->p_out, Tb, Lb, a0, c->d_mie,
                                                     c->d_dnorm, S->tgt, S->w, wpart);
    SHIP(hipGetLastError());
    std::vector<double> wp(M);
    SHIP(hipMemcpyAsync(wp.data(), wpart, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    SHIP(hipStreamSynchronize(s));
    double tot = 0.0;
    for (double v : wp) tot += v;
    S->wnorm = tot > 0 ? tot : 1.0;
    S->has_target = true;
  }
  SHIP(hipStreamSynchronize(s));
#undef SHIP
  if (a0_out)
    *a0_out = a0;
  else
    hipFree(a0);
  if (Tb) hipFree(Tb);
  if (Lb) hipFree(Lb);
  if (wpart) hipFree(wpart);
  return GRT_OK;
}

const uint16_t* W(grt_nn* n, int t) { return n->pb + n->off[t]; }
float* G(grt_nn* n, int t) { return n->g + n->off[t]; }

void forward(grt_nn* n, const Sample& S, hipStream_t s) {
  const int M = S.M, H = n->H, L = n->L, K = n->K, O = n->O;
  const int64_t ldz = 2 * H;
  float* Z0 = n->Z;
  gemm<uint16_t, EPI_BIAS_RELU>(s, M, H, NF, S.feat, NF, 1, W(n, T_WIN()), 1, NF, n->pre0, H, 1.f,
                                0.f, W(n, T_BIN()), Z0, ldz);
  for (int l = 0; l < L; ++l) {
    float* Zl = n->Z + (size_t)l * n->cap * ldz;
    float* Pl = n->Pb + (size_t)l * n->cap * H;
    float* Ql = n->Qb + (size_t)l * n->cap * H;
    float* Ul = n->upre + (size_t)l * n->cap * H;
    gemm<uint16_t, EPI_PLAIN>(s, M, H, H, Zl, ldz, 1, W(n, T_A(l)), 1, H, Pl, H);
    gemm<uint16_t, EPI_PLAIN>(s, M, H, H, Zl, ldz, 1, W(n, T_B(l)), 1, H, Ql, H);
    edge_fwd_kernel<<<M, std::max(64, H), 0, s>>>(H, K, S.nbr, S.cnt, S.edge, Pl, Ql, W(n, T_C(l)),
                                                  W(n, T_c(l)), Zl, ldz);
    float* next = (l + 1 < L) ? n->Z + (size_t)(l + 1) * n->cap * ldz : n->hL;
    const int64_t ldn = (l + 1 < L) ? ldz : H;
    gemm<uint16_t, EPI_BIAS_RESID>(s, M, H, 2 * H, Zl, ldz, 1, W(n, T_U(l)), 1, 2 * H, Ul, H, 1.f,
                                   0.f, W(n, T_u(l)), next, ldn, Zl, ldz);
  }
  gemm<uint16_t, EPI_BIAS>(s, M, O, H, n->hL, H, 1, W(n, T_WOUT(L)), 1, H, n->out, O, 1.f, 0.f,
                           W(n, T_BOUT(L)));
}

// loss into *loss_dst (device) and the gradient of every weight into n->g
void backward(grt_nn* n, const Sample& S, hipStream_t s, double* loss_dst) {
  const int M = S.M, H = n->H, L = n->L, K = n->K, O = n->O;
  const int64_t ldz = 2 * H;
  const int64_t no = (int64_t)M * O;
  const unsigned nlb = blocks_for(no, 256);
  loss_kernel<<<nlb, 256, 0, s>>>(no, n->out, S.tgt, S.w, 1.0 / S.wnorm, n->dout, n->lpart);
  loss_finish_kernel<<<1, 64, 0, s>>>((int)nlb, n->lpart, 1.0 / S.wnorm, loss_dst);
  // output layer
  gemm<float, EPI_PLAIN>(s, O, H, M, n->dout, 1, O, n->hL, H, 1, G(n, T_WOUT(L)), H);
  colsum_kernel<<<blocks_for(O, 64), 64, 0, s>>>(M, O, n->dout, O, G(n, T_BOUT(L)));
  gemm<uint16_t, EPI_PLAIN>(s, M, H, O, n->dout, O, 1, W(n, T_WOUT(L)), H, 1, n->dh, H);
  const unsigned nbh = blocks_for((int64_t)M * H, 256);
  for (int l = L - 1; l >= 0; --l) {
    float* Zl = n->Z + (size_t)l * n->cap * ldz;
    float* Pl = n->Pb + (size_t)l * n->cap * H;
    float* Ql = n->Qb + (size_t)l * n->cap * H;
    float* Ul = n->upre + (size_t)l * n->cap * H;
    relu_mask_kernel<<<nbh, 256, 0, s>>>(M, H, n->dh, H, Ul, H, n->dtmp, H);
    gemm<float, EPI_PLAIN>(s, H, 2 * H, M, n->dtmp, 1, H, Zl, ldz, 1, G(n, T_U(l)), 2 * H);
    colsum_kernel<<<blocks_for(H, 64), 64, 0, s>>>(M, H, n->dtmp, H, G(n, T_u(l)));
    gemm<uint16_t, EPI_PLAIN>(s, M, 2 * H, H, n->dtmp, H, 1, W(n, T_U(l)), 2 * H, 1, n->dz, ldz);
    add_kernel<<<nbh, 256, 0, s>>>(M, H, n->dz, ldz, n->dh, H);
    edge_bwd_kernel<<<M, std::max(64, H), 0, s>>>(H, K, S.nbr, S.cnt, S.edge, Pl, Ql, W(n, T_C(l)),
                                                  W(n, T_c(l)), n->dz, ldz, n->dP, n->part);
    edge_bwd_q_kernel<<<M, std::max(64, H), 0, s>>>(H, K, S.rev_off, S.rev, S.cnt, S.edge, Pl, Ql,
                                                    W(n, T_C(l)), W(n, T_c(l)), n->dz, ldz, n->dQ);
    colsum_kernel<<<blocks_for((int64_t)H * (NE + 1), 64), 64, 0, s>>>(M, H * (NE + 1), n->part,
                                                                       H * (NE + 1), n->red);
    split_partials_kernel<<<blocks_for(H, 64), 64, 0, s>>>(H, n->red, G(n, T_C(l)), G(n, T_c(l)));
    gemm<float, EPI_PLAIN>(s, H, H, M, n->dP, 1, H, Zl, ldz, 1, G(n, T_A(l)), H);
    gemm<float, EPI_PLAIN>(s, H, H, M, n->dQ, 1, H, Zl, ldz, 1, G(n, T_B(l)), H);
    gemm<uint16_t, EPI_PLAIN>(s, M, H, H, n->dP, H, 1, W(n, T_A(l)), H, 1, n->dh, H, 1.f, 1.f);
    gemm<uint16_t, EPI_PLAIN>(s, M, H, H, n->dQ, H, 1, W(n, T_B(l)), H, 1, n->dh, H, 1.f, 1.f);
  }
  relu_mask_kernel<<<nbh, 256, 0, s>>>(M, H, n->dh, H, n->pre0, H, n->dtmp, H);
  gemm<float, EPI_PLAIN>(s, H, NF, M, n->dtmp, 1, H, S.feat, NF, 1, G(n, T_WIN()), NF);
  colsum_kernel<<<blocks_for(H, 64), 64, 0, s>>>(M, H, n->dtmp, H, G(n, T_BIN()));
}

grt_status check_sample(grt_nn* n, int id, bool need_target) {
  if (id < 0 || id >= (int)n->samples.size() || n->samples[id].M == 0)
    return nset(n, GRT_EINVAL, "no such sample");
  if (need_target && !n->samples[id].has_target)
    return nset(n, GRT_ESTATE, "sample has no target");
  return GRT_OK;
}

}  // namespace

extern "C" {

grt_status grt_nn_create(grt_nn** out, int device, void* hip_stream, const grt_nn_config* cfg) {
  if (!out || !cfg) return GRT_EINVAL;
  *out = nullptr;
  if (cfg->width < 64 || cfg->width > 256 || cfg->width % 64 || cfg->layers < 1 ||
      cfg->layers > 8 || cfg->k < 1 || cfg->k > KMAX || cfg->p_out < 0 || cfg->p_out > 20)
    return GRT_EINVAL;
  grt_nn* n = new (std::nothrow) grt_nn();
  if (!n) return GRT_ENOMEM;
  n->device = device;
  n->H = cfg->width;
  n->L = cfg->layers;
  n->K = cfg->k;
  n->p_out = cfg->p_out;
  n->O = 2 * (2 * cfg->p_out + 1);
  const int64_t H = n->H;
  std::vector<int64_t> sizes = {H * NF, H};
  for (int l = 0; l < n->L; ++l) sizes.insert(sizes.end(), {H * H, H * H, H * NE, H, H * 2 * H, H});
  sizes.push_back((int64_t)n->O * H);
  sizes.push_back(n->O);
  int64_t o = 0;
  for (int64_t sz : sizes) {
    n->off.push_back(o);
    o += sz;
  }
  n->np = o;
  if (hipSetDevice(device) != hipSuccess) {
    delete n;
    return GRT_EHIP;
  }
  if (hip_stream) {
    n->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) {
      delete n;
      return GRT_EHIP;
    }
    n->own_stream = true;
  }
  bool ok = hipMalloc(&n->p, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->g, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->m1, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->m2, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->pb, sizeof(uint16_t) * o) == hipSuccess &&
            hipMemset(n->p, 0, sizeof(float) * o) == hipSuccess &&
            hipMemset(n->g, 0, sizeof(float) * o) == hipSuccess &&
            hipMemset(n->m1, 0, sizeof(float) * o) == hipSuccess &&
            hipMemset(n->m2, 0, sizeof(float) * o) == hipSuccess &&
            hipMemset(n->pb, 0, sizeof(uint16_t) * o) == hipSuccess;
  if (!ok) {
    grt_nn_destroy(n);
    return GRT_ENOMEM;
  }
  *out = n;
  return GRT_OK;
}

grt_status grt_nn_destroy(grt_nn* n) {
  if (!n) return GRT_OK;
  hipSetDevice(n->device);
  if (n->stream) hipStreamSynchronize(n->stream);
  for (auto& S : n->samples) S.release();
  void* p[] = {n->p, n->g, n->m1, n->m2, n->pb, n->pre0, n->Z, n->hL, n->Pb, n->Qb, n->upre,
               n->out, n->dout, n->dh, n->dz, n->dP, n->dQ, n->dtmp, n->part, n->red, n->lpart,
               n->losses};
  for (void* q : p)
    if (q) hipFree(q);
  if (n->own_stream) hipStreamDestroy(n->stream);
  delete n;
  return GRT_OK;
}

const char* grt_nn_error_message(const grt_nn* n) { return n ? n->err.c_str() : "null network"; }

grt_status grt_nn_num_params(const grt_nn* n, int64_t* np) {
  if (!n || !np) return GRT_EINVAL;
  *np = n->np;
  return GRT_OK;
}

grt_status grt_nn_set_params(grt_nn* n, const float* host, int64_t count) {
  if (!n || !host) return GRT_EINVAL;
  if (count != n->np) return nset(n, GRT_EINVAL, "parameter count mismatch");
  NNHIP(n, hipSetDevice(n->device));
  NNHIP(n, hipMemcpyAsync(n->p, host, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
  NNHIP(n, hipMemsetAsync(n->m1, 0, sizeof(float) * count, n->stream));
  NNHIP(n, hipMemsetAsync(n->m2, 0, sizeof(float) * count, n->stream));
  round_bf16_kernel<<<blocks_for(count, 256), 256, 0, n->stream>>>(count, n->p, n->pb);
  NNHIP(n, hipGetLastError());
  NNHIP(n, hipStreamSynchronize(n->stream));
  n->t_adam = 0;
  return GRT_OK;
}

grt_status grt_nn_get_params(grt_nn* n, float* host, int64_t count) {
  if (!n || !host) return GRT_EINVAL;
  if (count != n->np) return nset(n, GRT_EINVAL, "parameter count mismatch");
  NNHIP(n, hipSetDevice(n->device));
  NNHIP(n, hipMemcpyAsync(host, n->p, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
  NNHIP(n, hipStreamSynchronize(n->stream));
  return GRT_OK;
}

grt_status grt_nn_add_sample(grt_nn* n, grt_ctx* c, const void* beta_dev, int* id) {
  if (c && c->n_rhs > 1) return GRT_EUNSUP;   // one angle per sample / prediction
  if (c && has_shapes(c)) return GRT_EUNSUP;  // node features hold the Mie diagonal
  if (c && c->lossy) return GRT_EUNSUP;       // and real indices
  if (!n || !c || !id) return GRT_EINVAL;
  if (!c->built || c->M == 0 || c->device != n->device)
    return nset(n, GRT_ESTATE, "context not built, without inclusions, or on another device");
  NNHIP(n, hipSetDevice(n->device));
  Sample S;
  NNTRY(build_sample(n, c, static_cast<const cd*>(beta_dev), &S));
  n->samples.push_back(S);
  *id = (int)n->samples.size() - 1;
  return GRT_OK;
}

grt_status grt_nn_clear_samples(grt_nn* n) {
  if (!n) return GRT_EINVAL;
  hipSetDevice(n->device);
  hipStreamSynchronize(n->stream);
  for (auto& S : n->samples) S.release();
  n->samples.clear();
  return GRT_OK;
}

grt_status grt_nn_sample_size(grt_nn* n, int id, int64_t* M) {
  if (!n || !M) return GRT_EINVAL;
  NNTRY(check_sample(n, id, false));
  *M = n->samples[id].M;
  return GRT_OK;
}

grt_status grt_nn_get_sample(grt_nn* n, int id, float* feat, int* nbr, float* edge, float* target,
                             float* weight, double* wnorm) {
  if (!n) return GRT_EINVAL;
  NNTRY(check_sample(n, id, false));
  const Sample& S = n->samples[id];
  const size_t M = S.M, K = n->K, O = n->O;
  NNHIP(n, hipSetDevice(n->device));
  if (feat) NNHIP(n, hipMemcpy(feat, S.feat, sizeof(float) * M * NF, hipMemcpyDeviceToHost));
  if (nbr) NNHIP(n, hipMemcpy(nbr, S.nbr, sizeof(int) * M * K, hipMemcpyDeviceToHost));
  if (edge) NNHIP(n, hipMemcpy(edge, S.edge, sizeof(float) * M * K * NE, hipMemcpyDeviceToHost));
  if (target) NNHIP(n, hipMemcpy(target, S.tgt, sizeof(float) * M * O, hipMemcpyDeviceToHost));
  if (weight) NNHIP(n, hipMemcpy(weight, S.w, sizeof(float) * M * O, hipMemcpyDeviceToHost));
  if (wnorm) *wnorm = S.wnorm;
  return GRT_OK;
}

grt_status grt_nn_set_target(grt_nn* n, int id, const float* target, const float* weight,
                             double wnorm) {
  if (!n || !target || !weight || !(wnorm > 0)) return GRT_EINVAL;
  NNTRY(check_sample(n, id, false));
  Sample& S = n->samples[id];
  const size_t MO = (size_t)S.M * n->O;
  NNHIP(n, hipSetDevice(n->device));
  NNHIP(n, hipMemcpy(S.tgt, target, sizeof(float) * MO, hipMemcpyHostToDevice));
  NNHIP(n, hipMemcpy(S.w, weight, sizeof(float) * MO, hipMemcpyHostToDevice));
  S.wnorm = wnorm;
  S.has_target = true;
  return GRT_OK;
}

grt_status grt_nn_loss_grad(grt_nn* n, int id, double* loss, float* grad_host, float* out_host) {
  if (!n) return GRT_EINVAL;
  NNTRY(check_sample(n, id, true));
  const Sample& S = n->samples[id];
  NNHIP(n, hipSetDevice(n->device));
  NNTRY(ensure_cap(n, S.M));
  if (n->losses_cap < 1) {
    NNHIP(n, hipMalloc(&n->losses, sizeof(double) * 1024));
    n->losses_cap = 1024;
  }
  forward(n, S, n->stream);
  backward(n, S, n->stream, n->losses);
  NNHIP(n, hipGetLastError());
  if (loss) NNHIP(n, hipMemcpyAsync(loss, n->losses, sizeof(double), hipMemcpyDeviceToHost, n->stream));
  if (grad_host)
    NNHIP(n, hipMemcpyAsync(grad_host, n->g, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
  if (out_host)
    NNHIP(n, hipMemcpyAsync(out_host, n->out, sizeof(float) * (size_t)S.M * n->O,
                            hipMemcpyDeviceToHost, n->stream));
  NNHIP(n, hipStreamSynchronize(n->stream));
  return GRT_OK;
}

grt_status grt_nn_train(grt_nn* n, int64_t n_ids, const int* ids, int epochs, float lr, uint64_t seed,
                        double* last_epoch_loss) {
  if (!n || !ids || n_ids <= 0 || epochs < 1 || !(lr > 0)) return GRT_EINVAL;
  int maxM = 0;
  for (int64_t i = 0; i < n_ids; ++i) {
    NNTRY(check_sample(n, ids[i], true));
    maxM = std::max(maxM, n->samples[ids[i]].M);
  }
  NNHIP(n, hipSetDevice(n->device));
  NNTRY(ensure_cap(n, maxM));
  if (n->losses_cap < n_ids) {
    if (n->losses) hipFree(n->losses);
    n->losses = nullptr;
    NNHIP(n, hipMalloc(&n->losses, sizeof(double) * n_ids));
    n->losses_cap = (int)n_ids;
  }
  std::vector<int> order(ids, ids + n_ids);
  std::mt19937_64 rng(seed);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t i = n_ids - 1; i > 0; --i) {  // Fisher-Yates
      const int64_t r = (int64_t)(rng() % (uint64_t)(i + 1));
      std::swap(order[i], order[r]);
    }
    for (int64_t i = 0; i < n_ids; ++i) {
      const Sample& S = n->samples[order[i]];
      forward(n, S, n->stream);
      backward(n, S, n->stream, n->losses + i);
      ++n->t_adam;
      const float c1 = 1.f - std::pow(b1, (float)n->t_adam);
      const float c2 = 1.f - std::pow(b2, (float)n->t_adam);
      adam_kernel<<<blocks_for(n->np, 256), 256, 0, n->stream>>>(n->np, n->p, n->g, n->m1, n->m2,
                                                                 n->pb, lr, b1, b2, eps, c1, c2);
    }
    NNHIP(n, hipGetLastError());
  }
  std::vector<double> ls(n_ids);
  NNHIP(n, hipMemcpyAsync(ls.data(), n->losses, sizeof(double) * n_ids, hipMemcpyDeviceToHost,
                          n->stream));
  NNHIP(n, hipStreamSynchronize(n->stream));
  if (last_epoch_loss) {
    double s = 0.0;
    for (double v : ls) s += v;
    *last_epoch_loss = s / (double)n_ids;
  }
  return GRT_OK;
}

grt_status grt_nn_predict(grt_nn* n, grt_ctx* c, void* beta0_dev) {
  if (c && c->n_rhs > 1) return GRT_EUNSUP;   // one angle per sample / prediction
  if (c && has_shapes(c)) return GRT_EUNSUP;  // node features hold the Mie diagonal
  if (c && c->lossy) return GRT_EUNSUP;       // and real indices
  if (!n || !c || !beta0_dev) return GRT_EINVAL;
  if (!c->built || c->M == 0 || c->device != n->device)
    return nset(n, GRT_ESTATE, "context not built, without inclusions, or on another device");
  NNHIP(n, hipSetDevice(n->device));
  NNHIP(n, hipStreamSynchronize(n->stream));  // the workspace is shared with training
  NNTRY(ensure_cap(n, (int)c->M));
  Sample S;
  cd* a0 = nullptr;
  NNTRY(build_sample(n, c, nullptr, &S, &a0));
  hipStream_t s = c->stream;
  grt_status st = GRT_OK;
  forward(n, S, s);
  warm_kernel<<<blocks_for(c->n_beta, 256), 256, 0, s>>>((int)c->M, c->P, n->p_out, c->d_mie, a0,
                                                         n->out, static_cast<cd*>(beta0_dev));
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    st = nset(n, GRT_EHIP, "warm-start kernels failed");
  hipFree(a0);
  S.release();
  return st;
}

}  // extern "C"
