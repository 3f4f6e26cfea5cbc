// Restarted GMRES on the device for K beta = b (paper sec. 5: the preconditioned
// Schur system is solved iteratively by GMRES; sec. 6 reports its relative residual
// as the "GMRES error").  FP64 throughout: classical Gram-Schmidt applied twice
// (CGS2) for the Arnoldi basis on the device; each new Hessenberg column (j+2
// numbers) is copied to pinned host memory, where the complex Givens rotations,
// the residual estimate and, at the end of a cycle, the triangular solve run,
// one Arnoldi step behind the device so the GPU queue never drains.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "grt_internal.h"

namespace {

constexpr int KT = 256;
constexpr int NBLK_MAX = 16;  // most partial sums per dot product (ensure_workspace)

// sum_{b < nblk} p[b * stride] in the order b = 0, 1, ...; all loads are issued
// before the first add (nblk <= NBLK_MAX), so the sum costs one memory latency
template <typename T>
__device__ __forceinline__ T sum_partials(const T* p, size_t stride, int nblk) {
  T v[NBLK_MAX];
#pragma unroll
  for (int b = 0; b < NBLK_MAX; ++b) v[b] = b < nblk ? p[(size_t)b * stride] : T{};
  T s = v[0];
#pragma unroll
  for (int b = 1; b < NBLK_MAX; ++b)
    if (b < nblk) s += v[b];
  return s;
}

// partial[v][blk] = sum_{i in slice blk} conj(V_v[i]) w[i]
__global__ void __launch_bounds__(KT) dots_kernel(const cd* __restrict__ V, size_t ldv,
                                                   const cd* __restrict__ w, int n, cd* partial,
                                                   int nblk) {
  int v = blockIdx.y;
  const cd* a = V + (size_t)v * ldv;
  double sr = 0.0, si = 0.0;
  for (int i = blockIdx.x * KT + threadIdx.x; i < n; i += nblk * KT) {
    cd x = a[i], y = w[i];
    sr = fma(x.r, y.r, sr);
    sr = fma(x.i, y.i, sr);
    si = fma(x.r, y.i, si);
    si = fma(-x.i, y.r, si);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  __shared__ double rr[KT / 64], ri[KT / 64];
  int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { rr[wv] = sr; ri[wv] = si; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int t = 0; t < KT / 64; ++t) { a0 += rr[t]; a1 += ri[t]; }
    partial[(size_t)v * nblk + blockIdx.x] = cd{a0, a1};
  }
}

// h[v] = sum_b partial[v][b] (fixed order), then w[i] -= sum_v h[v] V_v[i].
// Every block redoes the small reduction; block 0 also stores h into the
// Hessenberg column (pass 0) or adds it (pass 1: the re-orthogonalisation).
// With npart given, block b also stores npart[b] = sum of |w_new[i]|^2 over its
// entries, the partial sums of the new direction's norm.
__global__ void __launch_bounds__(KT) update_kernel(const cd* __restrict__ V, size_t ldv, cd* w,
                                                     int n, const cd* __restrict__ partial,
                                                     int nblk, int nvec, cd* hcol, int pass,
                                                     double* npart) {
  __shared__ cd h[1024];
  for (int v = threadIdx.x; v < nvec; v += KT) {
    const cd s = sum_partials(partial + (size_t)v * nblk, 1, nblk);
    h[v] = s;
    if (blockIdx.x == 0) hcol[v] = pass ? hcol[v] + s : s;
  }
  __syncthreads();
  int i = blockIdx.x * KT + threadIdx.x;
  double s2 = 0.0;
  if (i < n) {
    cd acc = w[i];
    for (int v = 0; v < nvec; ++v) {
      cd hv = h[v];
      cd a = V[(size_t)v * ldv + i];
      acc.r -= hv.r * a.r - hv.i * a.i;
      acc.i -= hv.r * a.i + hv.i * a.r;
    }
    w[i] = acc;
    s2 = cabs2(acc);
  }
  if (!npart) return;  // uniform over the block
  for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
  __shared__ double r[KT / 64];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int t = 0; t < KT / 64; ++t) a += r[t];
    npart[blockIdx.x] = a;
  }
}

// sum_{b < np} p[b] in a fixed order (strided per thread, butterfly over the wave,
// waves in order); every thread of every block gets the same value.
__device__ __forceinline__ double block_sum(const double* p, int np) {
  double s = 0.0;
  for (int b = threadIdx.x; b < np; b += KT) s += p[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double r[KT / 64];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = s;
  __syncthreads();
  double a = 0.0;
  for (int t = 0; t < KT / 64; ++t) a += r[t];
  return a;
}

// sum |w|^2 partials
__global__ void __launch_bounds__(KT) norm2_kernel(const cd* __restrict__ w, int n, double* partial,
                                                    int nblk) {
  double s = 0.0;
  for (int i = blockIdx.x * KT + threadIdx.x; i < n; i += nblk * KT) s += cabs2(w[i]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double r[KT / 64];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int t = 0; t < KT / 64; ++t) a += r[t];
    partial[blockIdx.x] = a;
  }
}

__global__ void norm_finish_kernel(const double* partial, int nblk, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[b];
  *out = sqrt(s);
}

// dst = src * (1 / *nrm)   (dst may alias src)
__global__ void scale_kernel(const cd* src, cd* dst, int n, const double* nrm) {
  int i = blockIdx.x * KT + threadIdx.x;
  if (i >= n) return;
  double s = *nrm;
  dst[i] = (s > 0) ? (1.0 / s) * src[i] : src[i];
}

__global__ void sub_vec_kernel(const cd* a, const cd* b, cd* o, int n) {
  int i = blockIdx.x * KT + threadIdx.x;
  if (i < n) o[i] = a[i] - b[i];
}

__global__ void axpy_basis_kernel(cd* x, const cd* __restrict__ V, size_t ldv, int n,
                                  const cd* __restrict__ y, int k) {
  int i = blockIdx.x * KT + threadIdx.x;
  if (i >= n) return;
  cd acc = x[i];
  for (int v = 0; v < k; ++v) cmac(acc, y[v], V[(size_t)v * ldv + i]);
  x[i] = acc;
}

// vout = w / ||w|| with ||w|| from the np norm partials (every block redoes the
// short sum in the same order); block 0 also stores it as H[j+1][j] = hcol[j+1] and
// copies the finished column hcol[0..j+1] to the host mirror hhost.  xpre = dinv o
// vout (the unnormalised input of the next apply).
__global__ void __launch_bounds__(KT) norm_scale_kernel(const cd* w, cd* vout, int n,
                                                         const double* npart, int np, cd* hcol,
                                                         int j, cd* hhost, const double* dinv,
                                                         cd* xpre) {
  const double hn = sqrt(block_sum(npart, np));
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t <= j; t += KT) hhost[t] = hcol[t];
    if (threadIdx.x == 0) {
      hcol[j + 1] = cd{hn, 0.0};
      hhost[j + 1] = cd{hn, 0.0};
    }
  }
  int i = blockIdx.x * KT + threadIdx.x;
  if (i >= n) return;
  const cd v = hn > 0 ? (1.0 / hn) * w[i] : w[i];
  vout[i] = v;
  xpre[i] = dinv[i] * v;
}

}  // namespace

void graph_reset(grt_ctx* c) {
  for (hipGraphExec_t& g : c->graph_exec)
    if (g) {
      hipGraphExecDestroy(g);
      g = nullptr;
    }
}

static grt_status ensure_workspace(grt_ctx* c, int m) {
  if (c->krylov_restart == m && c->d_V) return GRT_OK;
  hipFree(c->d_V); hipFree(c->d_H);
  hipFree(c->d_y); hipFree(c->d_scal); hipFree(c->d_dotpart);
  const size_t n = (size_t)c->n_beta;
  c->n_dot_blocks = (int)std::min<size_t>(NBLK_MAX, (n + KT * 4 - 1) / (KT * 4));
  if (c->n_dot_blocks < 1) c->n_dot_blocks = 1;
  graph_reset(c);  // captured applies point into the workspace
  GRT_HIP(c, hipMalloc(&c->d_V, sizeof(cd) * n * (m + 5)));
  c->d_wtmp = c->d_V + n * (m + 4);
  GRT_HIP(c, hipMalloc(&c->d_H, sizeof(cd) * (size_t)(m + 1) * (m + 1)));
  GRT_HIP(c, hipMalloc(&c->d_y, sizeof(cd) * (m + 1)));
  // scalars, then the norm partials: n_dot_blocks of them from norm2_kernel, or one
  // per KT entries from the update pass
  GRT_HIP(c, hipMalloc(&c->d_scal, sizeof(double) * (16 + std::max<size_t>(c->n_dot_blocks,
                                                                           (n + KT - 1) / KT))));
  if (!c->ev_res[0]) {
    GRT_HIP(c, hipEventCreateWithFlags(&c->ev_res[0], hipEventDisableTiming));
    GRT_HIP(c, hipEventCreateWithFlags(&c->ev_res[1], hipEventDisableTiming));
  }
  GRT_HIP(c, hipMalloc(&c->d_dotpart, sizeof(cd) * ((size_t)(m + 2) * c->n_dot_blocks + 2 * (size_t)(m + 2))));
  if (!c->h_pinned) GRT_HIP(c, hipHostMalloc(&c->h_pinned, sizeof(double) * 16));
  if (c->h_H) hipHostFree(c->h_H);
  c->h_H = nullptr;
  c->h_H_dev = nullptr;
  // host mirror of the Hessenberg columns, then y: (m+1)^2 + (m+1) complex
  // (coherent, so that the columns the normalisation kernel writes there are read by
  // the host once the step's event has completed)
  GRT_HIP(c, hipHostMalloc(&c->h_H, sizeof(cd) * ((size_t)(m + 1) * (m + 1) + (m + 1)),
                           hipHostMallocMapped | hipHostMallocCoherent));
  GRT_HIP(c, hipHostGetDevicePointer((void**)&c->h_H_dev, c->h_H, 0));
  c->krylov_restart = m;
  return GRT_OK;
}

static grt_status vec_norm(grt_ctx* c, const cd* w, int n, double* out_dev) {
  int nb = c->n_dot_blocks;
  double* part = c->d_scal + 16;
  norm2_kernel<<<nb, KT, 0, c->stream>>>(w, n, part, nb);
  norm_finish_kernel<<<1, 64, 0, c->stream>>>(part, nb, out_dev);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

static grt_status read_scalar(grt_ctx* c, const double* dev, double* host) {
  GRT_HIP(c, hipMemcpyAsync(c->h_pinned, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  *host = c->h_pinned[0];
  return GRT_OK;
}

#define GRT_TRY(x)                 \
  do {                             \
    grt_status s_ = (x);           \
    if (s_ != GRT_OK) return s_;   \
  } while (0)

__global__ void add_vec_kernel(cd* x, const cd* e, int n) {
  int i = blockIdx.x * KT + threadIdx.x;
  if (i < n) x[i] = x[i] + e[i];
}

typedef grt_status (*KOp)(grt_ctx*, const cd*, cd*, const double*);

// y = d o x (elementwise; y may alias x)
__global__ void dscale_kernel(const cd* x, const double* d, cd* y, int n) {
  int i = blockIdx.x * KT + threadIdx.x;
  if (i < n) y[i] = d[i] * x[i];
}

// The normalised operators D K D^{-1} (D = |H_|n|(k2 R_m)|, a diagonal similarity
// that keeps the reduced system well conditioned when high-order coefficients are
// tiny).  Every apply reads D^{-1} x from d_xtmp and writes D K D^{-1} x to d_wtmp,
// fixed buffers, so with use_graph the kernel sequence of one apply is captured once
// as a HIP graph (per operator) and replayed; the graphs are dropped whenever the
// apply's configuration changes (graph_reset).
static grt_status apply_step(grt_ctx* c, KOp op, bool use_graph) {
  if (!use_graph || c->prof) return op(c, c->d_xtmp, c->d_wtmp, c->d_dnorm);
  hipGraphExec_t* ge = (op == apply_K) ? &c->graph_exec[0] : &c->graph_exec[1];
  if (!*ge) {
    hipGraph_t gr = nullptr;
    GRT_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    grt_status st = op(c, c->d_xtmp, c->d_wtmp, c->d_dnorm);
    hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (st != GRT_OK || e != hipSuccess) {
      if (gr) hipGraphDestroy(gr);
      return st != GRT_OK ? st
                          : set_err(c, GRT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(ge, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (e != hipSuccess) {
      *ge = nullptr;
      return set_err(c, GRT_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
  }
  GRT_HIP(c, hipGraphLaunch(*ge, c->stream));
  return GRT_OK;
}

// d_wtmp = D K D^{-1} xh
static grt_status apply_hat(grt_ctx* c, KOp op, const cd* xh, bool use_graph) {
  const int n = (int)c->n_beta;
  dscale_kernel<<<(n + KT - 1) / KT, KT, 0, c->stream>>>(xh, c->d_dinv, c->d_xtmp, n);
  return apply_step(c, op, use_graph);
}

struct CoreResult {
  int iters = 0, cycles = 0;
  int fast_applies = 0;
  double rel = 1.0;
  bool converged = false;
  bool x0_rejected = false;
};

// Restarted GMRES for op(x) = b from the iterate in x (updated in place).  b must not
// live in basis slots 0..m.  Stops at ||b - op x|| <= tol ||b|| or after maxit steps.
// With fast set (relaxed inexact GMRES), an Arnoldi step whose latest residual
// estimate is at most fast_rel ||b|| applies fast instead of op; the residual at
// every restart, and so the stopping test, is always op's.
static grt_status gmres_core(grt_ctx* c, KOp op, const cd* bvec, cd* x, double tol, int maxit,
                             int m, CoreResult* res, bool guard_x0, bool use_graph,
                             KOp fast = nullptr, double fast_rel = 0.0) {
  const int n = (int)c->n_beta;
  hipStream_t s = c->stream;
  const size_t ldv = (size_t)n;
  cd* V = c->d_V;
  const int gridn = (n + KT - 1) / KT;
  const int nblk = c->n_dot_blocks;
  double* d_bn = c->d_scal + 0;
  double* d_beta = c->d_scal + 1;
  double* d_npart = c->d_scal + 16;
  GRT_TRY(vec_norm(c, bvec, n, d_bn));
  double bn = 0.0;
  GRT_TRY(read_scalar(c, d_bn, &bn));
  *res = CoreResult{};
  if (!(bn > 0)) {
    res->rel = 0.0;
    res->converged = true;
    return GRT_OK;
  }
  int total = 0;
  const int ldh = m + 1;
  cd* hH = c->h_H;                            // host mirror of H (column j at hH + j ldh)
  cd* hy = c->h_H + (size_t)ldh * ldh;        // least-squares solution
  std::vector<cd> cs(m + 1), sn(m + 1), g(m + 2);
  // Column jj of H arrived on the host: rotate it by the previous rotations, make
  // the rotation [[conj c, conj s], [-s, c]] (c = a/den, s = b/den) that zeroes
  // H[jj+1][jj], rotate g alongside; |g[jj+1]| is the residual norm of the
  // iterate that uses the first jj+1 basis vectors.
  auto givens = [&](int jj) {
    cd* h = hH + (size_t)jj * ldh;
    for (int i = 0; i < jj; ++i) {
      cd t = conj(cs[i]) * h[i] + conj(sn[i]) * h[i + 1];
      h[i + 1] = -(sn[i] * h[i]) + cs[i] * h[i + 1];
      h[i] = t;
    }
    cd a = h[jj], b = h[jj + 1];
    double den = std::sqrt(cabs2(a) + cabs2(b));
    cd cc = den > 0 ? (1.0 / den) * a : cd{1.0, 0.0};
    cd ss = den > 0 ? (1.0 / den) * b : cd{0.0, 0.0};
    cs[jj] = cc;
    sn[jj] = ss;
    h[jj] = cd{den, 0.0};
    h[jj + 1] = cd{0.0, 0.0};
    g[jj + 1] = -(ss * g[jj]);
    g[jj] = conj(cc) * g[jj];
    return std::sqrt(cabs2(g[jj + 1]));
  };
  while (true) {
    // r = b - op x into V_0
    GRT_TRY(apply_hat(c, op, x, use_graph));
    sub_vec_kernel<<<gridn, KT, 0, s>>>(bvec, c->d_wtmp, V, n);
    GRT_TRY(vec_norm(c, V, n, d_beta));
    double beta = 0.0;
    GRT_TRY(read_scalar(c, d_beta, &beta));
    res->rel = beta / bn;
    if (guard_x0 && res->cycles == 0 && !res->x0_rejected && res->rel >= 1.0) {
      // an initial guess no better than zero is dropped: restart from x = 0
      GRT_HIP(c, hipMemsetAsync(x, 0, sizeof(cd) * n, s));
      res->x0_rejected = true;
      continue;
    }
    if (res->rel <= tol) { res->converged = true; break; }
    if (total >= maxit) break;
    scale_kernel<<<gridn, KT, 0, s>>>(V, V, n, d_beta);
    std::fill(g.begin(), g.end(), cd{0.0, 0.0});
    g[0] = cd{beta, 0.0};
    // Arnoldi steps.  The host never waits on the step it just queued: column j
    // of H is copied back and rotated after step j+1 has been queued, so at most
    // one step is computed past convergence (and discarded: the least-squares
    // solve uses columns 0..k-1 only, which that step leaves intact).
    int k = 0;
    int queued = 0;
    bool conv = false;
    double est = res->rel;  // latest residual estimate known on the host (relative)
    for (int j = 0; j < m && total + queued < maxit; ++j) {
      cd* w = c->d_wtmp;  // the new direction; normalised into V_{j+1} below
      const bool use_fast = fast && est <= fast_rel;
      const KOp opj = use_fast ? fast : op;
      if (use_fast) ++res->fast_applies;
      // from the second step on, the previous step left D^{-1} V_j in d_xtmp
      if (j == 0)
        GRT_TRY(apply_hat(c, opj, V, use_graph));
      else
        GRT_TRY(apply_step(c, opj, use_graph));
      cd* hcol = c->d_H + (size_t)j * ldh;
      for (int pass = 0; pass < 2; ++pass) {
        dim3 gd(nblk, j + 1);
        dots_kernel<<<gd, KT, 0, s>>>(V, ldv, w, n, c->d_dotpart, nblk);
        // the second pass also leaves the partial sums of |w|^2
        update_kernel<<<gridn, KT, 0, s>>>(V, ldv, w, n, c->d_dotpart, nblk, j + 1, hcol, pass,
                                           pass ? d_npart : nullptr);
      }
      // the normalisation also puts column j of H (j+2 numbers) into the host mirror
      norm_scale_kernel<<<gridn, KT, 0, s>>>(w, V + (size_t)(j + 1) * ldv, n, d_npart, gridn,
                                             hcol, j, c->h_H_dev + (size_t)j * ldh, c->d_dinv,
                                             c->d_xtmp);
      GRT_HIP(c, hipGetLastError());
      GRT_HIP(c, hipEventRecord(c->ev_res[j & 1], s));
      ++queued;
      if (j >= 1) {
        GRT_HIP(c, hipEventSynchronize(c->ev_res[(j - 1) & 1]));
        est = givens(j - 1) / bn;
        if (est <= tol) { k = j; conv = true; break; }
      }
      k = j + 1;
    }
    if (!conv && k == queued && k > 0) {  // the last queued step has not been checked yet
      GRT_HIP(c, hipEventSynchronize(c->ev_res[(k - 1) & 1]));
      givens(k - 1);
    }
    total += k;
    // back substitution R y = g on the leading k x k triangle (host), then x += V y
    for (int i = k - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int t = i + 1; t < k; ++t) acc -= hH[(size_t)t * ldh + i] * hy[t];
      cd dd = hH[(size_t)i * ldh + i];
      hy[i] = (cabs2(dd) > 0) ? cdiv(acc, dd) : cd{0.0, 0.0};
    }
    GRT_HIP(c, hipMemcpyAsync(c->d_y, hy, sizeof(cd) * k, hipMemcpyHostToDevice, s));
    axpy_basis_kernel<<<gridn, KT, 0, s>>>(x, V, ldv, n, c->d_y, k);
    GRT_HIP(c, hipGetLastError());
    // the host y buffer is rewritten next cycle: wait for the copy to land
    GRT_HIP(c, hipStreamSynchronize(s));
    res->cycles += 1;
  }
  res->iters = total;
  return GRT_OK;
}

grt_status gmres_solve(grt_ctx* c, const grt_solve_opts* o, cd* x, grt_solve_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  const int n = (int)c->n_beta;
  const int m = std::max(1, std::min(o->restart > 0 ? o->restart : 100, 1000));
  const int maxit = o->maxit > 0 ? o->maxit : 1000;
  const double tol = o->tol > 0 ? o->tol : 1e-9;
  GRT_TRY(ensure_workspace(c, m));
  const bool graph = o->use_graph != 0;
  hipStream_t s = c->stream;
  const size_t ldv = (size_t)n;
  const int gridn = (n + KT - 1) / KT;
  cd* bvec = c->d_V + (size_t)(m + 1) * ldv;  // slot m+1: b
  cd* rvec = c->d_V + (size_t)(m + 2) * ldv;  // slot m+2: refinement residual
  cd* evec = c->d_V + (size_t)(m + 3) * ldv;  // slot m+3: refinement correction
  GRT_TRY(rhs_b(c, bvec));
  // work in normalised variables: b^ = D b, x^ = D x
  dscale_kernel<<<gridn, KT, 0, s>>>(bvec, c->d_dnorm, bvec, n);
  if (!o->use_x0)
    GRT_HIP(c, hipMemsetAsync(x, 0, sizeof(cd) * n, s));
  else
    dscale_kernel<<<gridn, KT, 0, s>>>(x, c->d_dnorm, x, n);
  *st = grt_solve_stats{};
  CoreResult r;
  if (o->precision == GRT_FP64 || o->precision == GRT_FP32_RELAXED) {
    const bool relax = o->precision == GRT_FP32_RELAXED;
    const double sw = o->inner_tol > 0 ? o->inner_tol : std::min(1e-2, 1e5 * tol);
    GRT_TRY(gmres_core(c, apply_K, bvec, x, tol, maxit, m, &r, o->use_x0 != 0, graph,
                       relax ? apply_K_mixed : nullptr, sw));
    st->x0_rejected = r.x0_rejected ? 1 : 0;
    st->iters = r.iters;
    st->cycles = r.cycles;
    st->rel_resid = r.rel;
    st->refine_steps = 0;
    st->fp32_applies = r.fast_applies;
  } else {
    // FP64 iterative refinement around the FP32-translation operator:
    //   r = b - K x (FP64), solve K32 e = r to inner_tol, x += e.
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-5;
    const int max_ref = o->max_refine > 0 ? o->max_refine : 10;
    double* d_bn = c->d_scal + 4;
    double* d_rn = c->d_scal + 5;
    GRT_TRY(vec_norm(c, bvec, n, d_bn));
    double bn = 0.0;
    GRT_TRY(read_scalar(c, d_bn, &bn));
    int total = 0, cycles = 0;
    double rel = 1.0;
    bool conv = false;
    for (int outer = 0; outer <= max_ref; ++outer) {
      GRT_TRY(apply_hat(c, apply_K, x, graph));
      sub_vec_kernel<<<gridn, KT, 0, s>>>(bvec, c->d_wtmp, rvec, n);
      GRT_TRY(vec_norm(c, rvec, n, d_rn));
      double rn = 0.0;
      GRT_TRY(read_scalar(c, d_rn, &rn));
      rel = bn > 0 ? rn / bn : 0.0;
      if (outer == 0 && o->use_x0 && rel >= 1.0) {
        // an initial guess no better than zero is dropped
        GRT_HIP(c, hipMemsetAsync(x, 0, sizeof(cd) * n, s));
        st->x0_rejected = 1;
        GRT_HIP(c, hipMemcpyAsync(rvec, bvec, sizeof(cd) * n, hipMemcpyDeviceToDevice, s));
        rel = 1.0;
      }
      st->refine_steps = outer;
      if (rel <= tol) { conv = true; break; }
      if (outer == max_ref || total >= maxit) break;
      GRT_HIP(c, hipMemsetAsync(evec, 0, sizeof(cd) * n, s));
      GRT_TRY(gmres_core(c, apply_K_mixed, rvec, evec, itol, maxit - total, m, &r, false, graph));
      total += r.iters;
      st->fp32_applies += r.iters + r.cycles;
      cycles += r.cycles;
      add_vec_kernel<<<gridn, KT, 0, s>>>(x, evec, n);
      GRT_HIP(c, hipGetLastError());
    }
    st->iters = total;
    st->cycles = cycles;
    st->rel_resid = rel;
    r.converged = conv;
  }
  // back to beta = D^{-1} x^
  dscale_kernel<<<gridn, KT, 0, s>>>(x, c->d_dinv, x, n);
  GRT_HIP(c, hipGetLastError());
  GRT_HIP(c, hipStreamSynchronize(s));
  st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return r.converged ? GRT_OK : set_err(c, GRT_ENOCONV, "GMRES did not reach the tolerance");
}
