// Scattering matrices of non-circular inclusions (paper sec. 4.1, eqs. intg1 and
// intg2 and the formula for s_ln; shapes of eq. par1), and the product of the
// block-diagonal scattering matrix with a vector in the apply.
//
// Inclusion m has the boundary gamma(t) = rho(t) (cos(t + rot), sin(t + rot)),
// rho = a1 + a2 cos(a3 t), t in [0, 2 pi), relative to its centre, outward normal
// n = (gamma_y', -gamma_x') / |gamma'|.  With G_k = (i/4) H_0(k |x - y|) and its
// single, double, adjoint and hypersingular layer operators S, D, N, T, the
// densities [mu; sigma] of the incoming wave J_n(k2 r) e^{in theta} solve
//
//     mu + (S_k2 - S_kp) sigma + (D_k2 - D_kp) mu = -u_inc,
//    -sigma + (N_k2 - N_kp) sigma + (T_k2 - T_kp) mu = -du_inc/dn,
//
// and s_ln = (i/4) int [J_l(k2|y|) e^{-il theta_y} sigma_n + dn_y(same) mu_n] ds_y
// (Graf's theorem for (i/4) H_0; the paper prints the integral without that factor).
//
// Discretisation: Kress' product quadrature for periodic kernels with a logarithmic
// singularity (Kress 1991; Colton and Kress, Inverse Acoustic and Electromagnetic
// Scattering Theory, sec. 3.5).  Each kernel difference is written
// K1 ln(4 sin^2((t - tau)/2)) + K2, K1 being the kernel with (i/4) H_m(kr) replaced
// by -(1/(4 pi)) J_m(kr); on Nb = 2q nodes t_j = j pi / q the weight of node j for
// target i is R_{(i-j) mod Nb} K1 + (pi/q) K2, times |gamma'(t_j)|, with
// R_m = -(2 pi / q) sum_{p=1}^{q-1} cos(p m pi / q) / p - (pi / q^2) cos(m pi).
// On the diagonal (from (i/4) H_0(kr) = -(1/(2 pi)) J_0(kr) ln r + an even series):
// S difference K2 = -ln(k2/kp) / (2 pi); D and N differences 0; T difference
// K1 = -a, K2 = -a - 2b - a ln|gamma'|^2, a = (k2^2 - kp^2) / (8 pi),
// b = -(i/16)(k2^2 - kp^2) + (k2^2 c(k2) - kp^2 c(kp)) / (8 pi) - (k2^2 - kp^2) / (8 pi),
// c(k) = ln(k/2) + Euler's gamma.
//
// The systems of a chunk of inclusions are assembled on the device, factorised and
// solved with rocSOLVER's batched LU, and reduced to the (2P+1)^2 blocks by a
// kernel; the blocks stay resident (d_sblk[m][l][n], l the output order).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dev_bessel.h"
#include "grt_internal.h"

namespace {

constexpr int SB_CHUNK = 256;   // inclusions whose systems are solved together

struct Node {
  double x, y, nx, ny, sp;
};

__device__ __forceinline__ Node shape_node(const double* sh, int j, int Nb) {
  const double a1 = sh[0], a2 = sh[1], a3 = sh[2], rot = sh[3];
  const double t = (2.0 * GRT_PI / Nb) * j;
  double st, ct, sa, ca;
  sincos(t + rot, &st, &ct);
  sincos(a3 * t, &sa, &ca);
  const double rho = a1 + a2 * ca, drho = -a2 * a3 * sa;
  const double dx = drho * ct - rho * st, dy = drho * st + rho * ct;
  const double sp = sqrt(dx * dx + dy * dy);
  return Node{rho * ct, rho * st, dy / sp, -dx / sp, sp};
}

// R_m of Kress' rule on Nb = 2q nodes, m = 0 .. Nb-1
__global__ void kress_weights_kernel(int Nb, double* R) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= Nb) return;
  const int q = Nb / 2;
  double s = 0.0;
  for (int p = 1; p < q; ++p) s += cos(p * m * GRT_PI / q) / p;
  R[m] = -(2.0 * GRT_PI / q) * s - (GRT_PI / ((double)q * q)) * ((m & 1) ? -1.0 : 1.0);
}

// The four kernels of wavenumber k between distinct nodes (values and ln|x-y|^2
// coefficients): out[0..3] = S, D, N, T and out1[0..3] their coefficients.
__device__ __forceinline__ void kernels(double k, double rx, double ry, double r, double rnx,
                                        double rny, double nxny, cd* out, double* out1) {
  const double z = k * r;
  double j[3], j0, j1, y0, y1;
  bessel01(z, j0, j1, y0, y1);
  bessel_jn_array(z, 2, j);
  const double y2 = 2.0 * y1 / z - y0;
  const cd H0{j[0], y0}, H1{j[1], y1}, H2{j[2], y2};
  const cd qi{0.0, 0.25};  // i/4
  out[0] = qi * H0;
  out[1] = (k * rny / r) * (qi * H1);
  out[2] = (-k * rnx / r) * (qi * H1);
  out[3] = k * (qi * ((-k * rnx * rny / (r * r)) * H2 + (nxny / r) * H1));
  const double c = -1.0 / (4.0 * GRT_PI);
  out1[0] = c * j[0];
  out1[1] = c * k * j[1] * rny / r;
  out1[2] = -c * k * j[1] * rnx / r;
  out1[3] = c * k * (-k * j[2] * rnx * rny / (r * r) + j[1] * nxny / r);
}

// A[m] (column-major, NN = 2 Nb): one thread per (target i, source j) of one
// inclusion; rows [intg1; intg2], columns [mu; sigma].
__global__ void bie_assemble_kernel(int m0, int Nb, const double* __restrict__ shape,
                                    double k2, const double* __restrict__ kp_all,
                                    const double* __restrict__ R, cd* A) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nb * Nb) return;
  const int i = e % Nb, j = e / Nb;
  const double* sh = shape + 4 * (size_t)(m0 + b);
  const double kp = kp_all[m0 + b];
  const int NN = 2 * Nb;
  cd* Am = A + (size_t)b * NN * NN;
  const Node X = shape_node(sh, i, Nb), Y = shape_node(sh, j, Nb);
  const double w = (2.0 * GRT_PI / Nb) * Y.sp;      // (pi / q) |gamma'(t_j)|
  const double Rw = R[(i - j + Nb) % Nb] * Y.sp;    // R_{i-j} |gamma'(t_j)|
  cd v[4];
  if (i != j) {
    const double rx = X.x - Y.x, ry = X.y - Y.y;
    const double r = sqrt(rx * rx + ry * ry);
    const double rnx = rx * X.nx + ry * X.ny, rny = rx * Y.nx + ry * Y.ny;
    const double nxny = X.nx * Y.nx + X.ny * Y.ny;
    cd ka[4], kb[4];
    double ka1[4], kb1[4];
    kernels(k2, rx, ry, r, rnx, rny, nxny, ka, ka1);
    kernels(kp, rx, ry, r, rnx, rny, nxny, kb, kb1);
    const double st = sin(GRT_PI * (i - j) / Nb);
    const double L = log(4.0 * st * st);
    for (int q = 0; q < 4; ++q) {
      const cd K = ka[q] - kb[q];
      const double K1 = ka1[q] - kb1[q];
      v[q] = Rw * cd{K1, 0.0} + w * (K - cd{K1 * L, 0.0});
    }
  } else {
    const double a = (k2 * k2 - kp * kp) / (8.0 * GRT_PI);
    const double cr = (k2 * k2 * (log(0.5 * k2) + GRT_EULER_GAMMA) -
                       kp * kp * (log(0.5 * kp) + GRT_EULER_GAMMA)) / (8.0 * GRT_PI) - a;
    const cd bb{cr, -(k2 * k2 - kp * kp) / 16.0};
    v[0] = cd{w * (-log(k2 / kp) / (2.0 * GRT_PI)), 0.0};
    v[1] = cd{0.0, 0.0};
    v[2] = cd{0.0, 0.0};
    // T: R_0 K1 + (pi/q) K2 with K1 = -a, K2 = -a - 2b - a ln|gamma'|^2
    const cd K2 = cd{-a - a * log(Y.sp * Y.sp), 0.0} - 2.0 * bb;
    v[3] = cd{-a * Rw, 0.0} + w * K2;
  }
  // [[I + D, S], [T, -I + N]]
  if (i == j) {
    v[1].r += 1.0;
    v[2].r -= 1.0;
  }
  Am[(size_t)j * NN + i] = v[1];               // D block: row i, column j (mu)
  Am[(size_t)(Nb + j) * NN + i] = v[0];        // S block: row i, column Nb + j (sigma)
  Am[(size_t)j * NN + Nb + i] = v[3];          // T block: row Nb + i, column j
  Am[(size_t)(Nb + j) * NN + Nb + i] = v[2];   // N block: row Nb + i, column Nb + j
}

// F_n(x) = J_n(k|x|) e^{in theta_x} for n = -(P+1) .. P+1 at a point (out[n + P + 1])
__device__ __forceinline__ void jwaves(double k, double x, double y, int P, cd* out,
                                       double* jbuf) {
  const double r = sqrt(x * x + y * y);
  const double th = atan2(y, x);
  bessel_jn_array(k * r, P + 1, jbuf);
  for (int n = 0; n <= P + 1; ++n) {
    double s, c;
    sincos(n * th, &s, &c);
    const cd fp{jbuf[n] * c, jbuf[n] * s};                 // J_n e^{in theta}
    const double sg = (n & 1) ? -1.0 : 1.0;                // J_{-n} = (-1)^n J_n
    out[P + 1 + n] = fp;
    out[P + 1 - n] = cd{sg * jbuf[n] * c, -sg * jbuf[n] * s};
  }
}

constexpr int SB_PMAX = 20;

// Right-hand sides (column-major [NN][nb]): column n: [-F_n; -dF_n/dn] at the nodes,
// (d_x, d_y) F_n = (k/2)(F_{n-1} - F_{n+1}, i (F_{n-1} + F_{n+1})).
__global__ void bie_rhs_kernel(int m0, int Nb, int P, const double* __restrict__ shape,
                               double k2, cd* B) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Nb) return;
  const int NN = 2 * Nb, nb = 2 * P + 1;
  const Node X = shape_node(shape + 4 * (size_t)(m0 + b), j, Nb);
  cd F[2 * SB_PMAX + 3];
  double jb[SB_PMAX + 2];
  jwaves(k2, X.x, X.y, P, F, jb);
  cd* Bm = B + (size_t)b * NN * nb;
  for (int c = 0; c < nb; ++c) {
    const int n = c - P;
    const cd fm = F[P + 1 + n - 1], fp = F[P + 1 + n + 1];
    const cd gx = (0.5 * k2) * (fm - fp);
    const cd gy = (0.5 * k2) * times_i(fm + fp);
    Bm[(size_t)c * NN + j] = -F[P + 1 + n];
    Bm[(size_t)c * NN + Nb + j] = -(X.nx * gx + X.ny * gy);
  }
}

// s_ln = (i/4) sum_j w_j [W_l sigma_n + dW_l/dn mu_n], W_l = J_l e^{-il theta} =
// (-1)^l F_{-l}; one thread per (l, n) of one inclusion.  X: solutions [NN][nb].
__global__ void sblock_kernel(int m0, int Nb, int P, const double* __restrict__ shape,
                              double k2, const cd* __restrict__ X, cd* sblk) {
  const int b = blockIdx.y;
  const int nb = 2 * P + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * nb) return;
  const int l = e / nb - P, n = e % nb;   // output order l, input column n
  const int NN = 2 * Nb;
  const double* sh = shape + 4 * (size_t)(m0 + b);
  const cd* Xm = X + (size_t)b * NN * nb + (size_t)n * NN;
  cd F[2 * SB_PMAX + 3];
  double jb[SB_PMAX + 2];
  cd acc{0.0, 0.0};
  const double sg = (l & 1) ? -1.0 : 1.0;
  for (int j = 0; j < Nb; ++j) {
    const Node Y = shape_node(sh, j, Nb);
    jwaves(k2, Y.x, Y.y, P, F, jb);
    const int o = -l;   // W_l = (-1)^l F_o
    const cd W = sg * F[P + 1 + o];
    const cd fm = F[P + 1 + o - 1], fp = F[P + 1 + o + 1];
    const cd gx = (0.5 * k2 * sg) * (fm - fp);
    const cd gy = (0.5 * k2 * sg) * times_i(fm + fp);
    const cd dW = Y.nx * gx + Y.ny * gy;
    const double w = (2.0 * GRT_PI / Nb) * Y.sp;
    acc += w * (W * Xm[Nb + j] + dW * Xm[j]);   // sigma at Nb + j, mu at j
  }
  sblk[((size_t)(m0 + b) * nb + (l + P)) * nb + n] = cd{0.0, 0.25} * acc;
}

// The product of the block-diagonal scattering matrix with w, one thread per entry
// (j, l): mode 0: y = x - S w; mode 1: y = S w; then y *= oscale when given.
__global__ void __launch_bounds__(256) sblock_apply_kernel(int M, int P, const cd* __restrict__ S,
                                                           const cd* __restrict__ x,
                                                           const cd* __restrict__ w, cd* y,
                                                           int mode,
                                                           const double* __restrict__ oscale) {
  const int nb = 2 * P + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * nb) return;
  const int64_t j = i / nb;
  const cd* row = S + (size_t)i * nb;
  const cd* wj = w + (size_t)j * nb;
  cd acc{0.0, 0.0};
  for (int n = 0; n < nb; ++n) cmac(acc, row[n], wj[n]);
  const cd v = mode == 0 ? x[i] - acc : acc;
  y[i] = oscale ? oscale[i] * v : v;
}

}  // namespace

bool has_shapes(const grt_ctx* c) { return !c->hshape.empty(); }

void launch_sblock_apply(grt_ctx* c, const cd* x, const cd* w, cd* y, int mode,
                         const double* oscale, hipStream_t s) {
  const int64_t n = c->n_beta;
  sblock_apply_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((int)c->M, c->P, c->d_sblk, x, w,
                                                                  y, mode, oscale);
}

static grt_status rs_err(grt_ctx* c, const char* what, rocblas_status s) {
  return set_err(c, GRT_EHIP, std::string(what) + " failed (rocblas status " +
                                  std::to_string((int)s) + ")");
}

// d_sblk[m] for every inclusion (inputs: the host shapes, d_kp on the device).
grt_status build_scattering_blocks(grt_ctx* c) {
  const int64_t M = c->M;
  const int P = c->P, nb = 2 * P + 1;
  const int Nb = c->shape_nodes, NN = 2 * Nb;
  hipStream_t s = c->stream;
  if (P > SB_PMAX) return set_err(c, GRT_EUNSUP, "non-circular inclusions need P <= 20");
  GRT_HIP(c, hipMalloc(&c->d_sblk, sizeof(cd) * (size_t)M * nb * nb));
  GRT_HIP(c, hipMalloc(&c->d_wS, sizeof(cd) * (size_t)c->n_beta));
  double *d_shape = nullptr, *d_R = nullptr;
  cd *A = nullptr, *B = nullptr;
  rocblas_int *ipiv = nullptr, *info = nullptr;
  const int chunk = (int)std::min<int64_t>(M, SB_CHUNK);
  GRT_HIP(c, hipMalloc(&d_shape, sizeof(double) * 4 * (size_t)M));
  GRT_HIP(c, hipMalloc(&d_R, sizeof(double) * Nb));
  GRT_HIP(c, hipMalloc(&A, sizeof(cd) * (size_t)chunk * NN * NN));
  GRT_HIP(c, hipMalloc(&B, sizeof(cd) * (size_t)chunk * NN * nb));
  GRT_HIP(c, hipMalloc(&ipiv, sizeof(rocblas_int) * (size_t)chunk * NN));
  GRT_HIP(c, hipMalloc(&info, sizeof(rocblas_int) * (size_t)chunk));
  GRT_HIP(c, hipMemcpyAsync(d_shape, c->hshape.data(), sizeof(double) * 4 * (size_t)M,
                            hipMemcpyHostToDevice, s));
  kress_weights_kernel<<<(Nb + 63) / 64, 64, 0, s>>>(Nb, d_R);
  rocblas_handle hb;
  rocblas_status rs = rocblas_create_handle(&hb);
  if (rs != rocblas_status_success) return rs_err(c, "rocblas_create_handle", rs);
  rocblas_set_stream(hb, s);
  grt_status st = GRT_OK;
  std::vector<rocblas_int> hinfo(chunk);
  for (int64_t m0 = 0; m0 < M && st == GRT_OK; m0 += chunk) {
    const int cnt = (int)std::min<int64_t>(chunk, M - m0);
    dim3 ga((unsigned)((Nb * Nb + 127) / 128), (unsigned)cnt);
    bie_assemble_kernel<<<ga, 128, 0, s>>>((int)m0, Nb, d_shape, c->g.k[1], c->d_kp, d_R, A);
    dim3 gr((unsigned)((Nb + 63) / 64), (unsigned)cnt);
    bie_rhs_kernel<<<gr, 64, 0, s>>>((int)m0, Nb, P, d_shape, c->g.k[1], B);
    if (hipGetLastError() != hipSuccess) {
      st = set_err(c, GRT_EHIP, "inclusion system kernels failed to launch");
      break;
    }
    auto* Ar = reinterpret_cast<rocblas_double_complex*>(A);
    auto* Br = reinterpret_cast<rocblas_double_complex*>(B);
    rs = rocsolver_zgetrf_strided_batched(hb, NN, NN, Ar, NN, (rocblas_stride)NN * NN, ipiv, NN,
                                          info, cnt);
    if (rs != rocblas_status_success) { st = rs_err(c, "rocsolver_zgetrf_strided_batched", rs); break; }
    rs = rocsolver_zgetrs_strided_batched(hb, rocblas_operation_none, NN, nb, Ar, NN,
                                          (rocblas_stride)NN * NN, ipiv, NN, Br, NN,
                                          (rocblas_stride)NN * nb, cnt);
    if (rs != rocblas_status_success) { st = rs_err(c, "rocsolver_zgetrs_strided_batched", rs); break; }
    dim3 gs((unsigned)((nb * nb + 63) / 64), (unsigned)cnt);
    sblock_kernel<<<gs, 64, 0, s>>>((int)m0, Nb, P, d_shape, c->g.k[1], B, c->d_sblk);
    if (hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * cnt, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = set_err(c, GRT_EHIP, "inclusion systems: synchronisation failed");
      break;
    }
    for (int q = 0; q < cnt; ++q)
      if (hinfo[q] != 0) {
        st = set_err(c, GRT_EGEOM, "the integral equation of inclusion " +
                                       std::to_string(m0 + q) + " is singular");
        break;
      }
  }
  rocblas_destroy_handle(hb);
  hipFree(d_shape);
  hipFree(d_R);
  hipFree(A);
  hipFree(B);
  hipFree(ipiv);
  hipFree(info);
  return st;
}
