// C ABI of the grating library: context, validation, orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "grt_internal.h"

grt_status set_err(grt_ctx* c, grt_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define GRT_CHECK_CTX(c)                   \
  do {                                     \
    if (!(c)) return GRT_EINVAL;           \
    (c)->err.clear();                      \
  } while (0)

namespace {

void free_all(grt_ctx* c) {
  graph_reset(c);
  ++c->gen;
  fmm_release(c);
  if (c->rhs_batch) {
    grt_batch_destroy(c->rhs_batch);
    c->rhs_batch = nullptr;
  }
  for (void* p : {(void*)c->d_blkX, (void*)c->d_blkY, (void*)c->d_blkph, (void*)c->d_blkw})
    if (p) hipFree(p);
  c->d_blkX = c->d_blkY = nullptr;
  c->d_blkph = nullptr;
  c->d_blkw = nullptr;
  c->blk_Rp = 0;
  if (c->lf) {  // layer-side buffers belong to the shared factors
    c->d_yw = c->d_colscale = c->d_sv = c->d_htab = c->d_node = nullptr;
    c->d_wcorr = c->d_A = c->d_U = c->d_VH = c->d_W1 = c->d_W2 = c->d_W3 = c->d_f = nullptr;
    c->lf.reset();
  }
  void* bufs[] = {c->d_cx, c->d_cy, c->d_rad, c->d_kp, c->d_kp_im, c->d_yw, c->d_node, c->d_wcorr, c->d_A,
                  c->d_colscale, c->d_sv, c->d_U, c->d_VH, c->d_W1, c->d_W2, c->d_W3,
                  c->d_mie, c->d_l2l, c->d_f, c->d_pT, c->d_pC, c->d_pB, c->d_pL,
                  c->d_gvec, c->d_tvec, c->d_wvec, c->d_V, c->d_H, c->d_htab,
                  c->d_y, c->d_scal, c->d_dotpart, c->d_x32, c->d_pT32,
                  c->d_pN, c->d_noff, c->d_nlist, c->d_dnorm, c->d_dinv, c->d_xtmp, c->d_ntgt, c->d_npart,
                  c->d_table, c->d_table32, c->d_sblk, c->d_wS};
  for (void* p : bufs)
    if (p) hipFree(p);
  c->d_cx = c->d_cy = c->d_rad = c->d_kp = c->d_yw = c->d_colscale = c->d_sv = c->d_scal =
      c->d_htab = c->d_node = c->d_kp_im = nullptr;
  c->d_wcorr = c->d_A = c->d_U = c->d_VH = c->d_W1 = c->d_W2 = c->d_W3 = c->d_mie = c->d_l2l =
      c->d_f = c->d_pT = c->d_pC = c->d_pB = c->d_pL = c->d_gvec = c->d_tvec = c->d_wvec =
          c->d_V = c->d_H = c->d_y = c->d_dotpart = nullptr;
  c->d_x32 = nullptr;
  c->d_pT32 = nullptr;
  c->d_pN = nullptr;
  c->d_noff = nullptr;
  c->d_nlist = nullptr;
  c->n_near = 0;
  c->d_dnorm = c->d_dinv = nullptr;
  c->d_xtmp = nullptr;
  c->d_ntgt = nullptr;
  c->d_npart = nullptr;
  c->d_table = nullptr;
  c->d_table32 = nullptr;
  c->d_sblk = nullptr;
  c->d_wS = nullptr;
  c->d_wtmp = nullptr;
  c->krylov_restart = 0;
  c->built = false;
  c->trans_built = false;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

// context of right-hand side r (r = 0: this one)
grt_ctx* rhs_ctx(grt_ctx* c, int64_t r) { return r == 0 ? c : c->rhs[(size_t)r - 1]; }

void destroy_rhs(grt_ctx* c, size_t keep) {
  while (c->rhs.size() > keep) {
    grt_destroy(c->rhs.back());
    c->rhs.pop_back();
  }
}

}  // namespace

extern "C" {

grt_status grt_create(grt_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return GRT_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GRT_EHIP;
  if (hip_device < 0 || hip_device >= ndev) return GRT_EINVAL;
  grt_ctx* c = new (std::nothrow) grt_ctx();
  if (!c) return GRT_ENOMEM;
  c->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    return GRT_EHIP;
  }
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GRT_EHIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return GRT_OK;
}

grt_status grt_destroy(grt_ctx* c) {
  if (!c) return GRT_OK;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  free_all(c);
  destroy_rhs(c, 0);
  for (hipEvent_t e : c->prof_ev) hipEventDestroy(e);
  for (hipEvent_t e : c->ev_res)
    if (e) hipEventDestroy(e);
  if (c->h_pinned) hipHostFree(c->h_pinned);
  if (c->h_H) hipHostFree(c->h_H);
  if (c->stream2) {
    hipStreamSynchronize(c->stream2);
    hipStreamDestroy(c->stream2);
  }
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
  return GRT_OK;
}

const char* grt_error_message(const grt_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

grt_status grt_set_problem(grt_ctx* c, const grt_layers* lay, const grt_inclusions* inc,
                           const grt_incidence* wave) {
  GRT_CHECK_CTX(c);
  if (!lay || !inc || !wave) return set_err(c, GRT_EINVAL, "null argument");
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  free_all(c);
  c->have_problem = false;
  const grt_layers& L = *lay;
  if (!finite_pos(L.d) || !finite_pos(L.h) || !(std::isfinite(L.y0) && L.y0 > L.h))
    return set_err(c, GRT_EINVAL, "need d > 0, h > 0, y0 > h");
  for (int l = 0; l < 3; ++l) {
    if (!finite_pos(L.n_layer[l])) return set_err(c, GRT_EINVAL, "layer indices must be > 0");
    if (L.Nw[l] < 1 || L.Nw[l] > 100000) return set_err(c, GRT_EINVAL, "bad wall node count");
    if (L.Q[l] < 0 || L.Q[l] > 400) return set_err(c, GRT_EINVAL, "J order Q must be in [0, 400]");
  }
  if (L.zeta_K < 1 || L.zeta_K > 16) return set_err(c, GRT_EINVAL, "zeta_K must be in [1, 16]");
  if (L.N < 2 * L.zeta_K + 1 || L.N > 1000000) return set_err(c, GRT_EINVAL, "N too small for the stencil");
  if (L.Nu < 1 || L.Nrb < 1 || L.Nrb > 100000) return set_err(c, GRT_EINVAL, "bad Nu / Nrb");
  if (!(L.pinv_eps > 0 && L.pinv_eps < 1)) return set_err(c, GRT_EINVAL, "pinv_eps must be in (0, 1)");
  if (L.n_fourier < 0 || L.n_fourier > 64)
    return set_err(c, GRT_EINVAL, "n_fourier must be in [0, 64]");
  if (L.n_fourier > 0 && !L.iface) return set_err(c, GRT_EINVAL, "n_fourier > 0 needs iface");
  const int F = L.n_fourier;
  std::vector<double> iface(L.iface ? L.iface : (const double*)nullptr,
                            L.iface ? L.iface + 4 * F : (const double*)nullptr);
  for (double v : iface)
    if (!std::isfinite(v)) return set_err(c, GRT_EINVAL, "non-finite interface coefficient");
  if (F > 0) {
    // the graphs keep their order and stay between Gamma_u and Gamma_d
    const int ns = 4096;
    for (int i = 0; i < ns; ++i) {
      const double x = -0.5 * L.d + (i + 0.5) * L.d / ns;
      const double f1 = iface_height(iface.data(), F, 0, L.h, L.d, x, 0);
      const double f2 = iface_height(iface.data(), F, 1, L.h, L.d, x, 0);
      if (!(f1 > f2 && f1 < L.y0 && f2 > -L.y0))
        return set_err(c, GRT_EINVAL, "curved interfaces must keep Gamma_1 above Gamma_2, "
                                      "both strictly between -y0 and y0");
    }
  }
  if (!finite_pos(wave->omega)) return set_err(c, GRT_EINVAL, "omega must be > 0");
  const int64_t R = wave->n_rhs > 1 ? wave->n_rhs : 1;
  if (wave->n_rhs < 0 || R > 65536) return set_err(c, GRT_EINVAL, "n_rhs must be in [0, 65536]");
  if (R > 1 && !wave->phis) return set_err(c, GRT_EINVAL, "n_rhs > 1 needs phis");
  const double phi0 = R > 1 ? wave->phis[0] : wave->phi;
  for (int64_t r = 0; r < R; ++r) {
    const double ph = R > 1 ? wave->phis[r] : wave->phi;
    if (!std::isfinite(ph) || std::fabs(ph) >= M_PI / 2)
      return set_err(c, GRT_EINVAL, "|phi| must be < pi/2");
  }
  if (wave->P < 1 || wave->P > 40) return set_err(c, GRT_EINVAL, "P must be in [1, 40]");
  if (wave->polarization != GRT_TM && wave->polarization != GRT_TE)
    return set_err(c, GRT_EINVAL, "polarization must be GRT_TM or GRT_TE");
  if (wave->polarization == GRT_TE && inc->shape && inc->M > 0)
    return set_err(c, GRT_EUNSUP, "non-circular inclusions are TM only");
  if (!std::isfinite(L.n3_im) || L.n3_im < 0)
    return set_err(c, GRT_EINVAL, "n3_im must be finite and >= 0");
  if (L.n3_im > 0) {
    if (L.n3_im > 0.1 * L.n_layer[2])
      return set_err(c, GRT_EUNSUP, "an absorbing substrate is taken for n3_im <= 0.1 n_3");
    // the bottom layer's J expansion about (0, -(h + y0) / 2) is evaluated up to the
    // corners of Gamma_d and the highest point of Gamma_2
    double hi = -L.h;
    for (int i = 0; F > 0 && i < 4096; ++i)
      hi = std::max(hi, iface_height(iface.data(), F, 1, L.h, L.d,
                                     -0.5 * L.d + (i + 0.5) * L.d / 4096, 0));
    const double reach = std::hypot(0.5 * L.d, std::max(hi + 0.5 * (L.h + L.y0),
                                                        0.5 * (L.y0 - L.h)));
    const double k3 = wave->omega * std::hypot(L.n_layer[2], L.n3_im);
    if (k3 * reach > 60.0)
      return set_err(c, GRT_EUNSUP, "absorbing substrate: |k_3| times the reach of its J "
                                    "expansion above 60");
  }
  if (!supported_P(wave->P)) return set_err(c, GRT_EUNSUP, "multipole order P not compiled in");
  const int64_t M = inc->M;
  if (M < 0 || M > 10000000) return set_err(c, GRT_EINVAL, "bad M");
  if (M > 0 && (!inc->x || !inc->y || !inc->radius || !inc->n_incl))
    return set_err(c, GRT_EINVAL, "null inclusion arrays");
  if (L.Q[1] + wave->P + 1 > 511) return set_err(c, GRT_EINVAL, "Q[1] + P too large");
  c->hx.assign(inc->x, inc->x + M);
  c->hy.assign(inc->y, inc->y + M);
  c->hr.assign(inc->radius, inc->radius + M);
  c->hn.assign(inc->n_incl, inc->n_incl + M);
  c->hshape.clear();
  c->shape_nodes = 0;
  c->hn_im.clear();
  c->lossy = false;
  if (inc->n_incl_im && M > 0) {
    for (int64_t m = 0; m < M; ++m) {
      const double v = inc->n_incl_im[m];
      if (!std::isfinite(v) || v < 0)
        return set_err(c, GRT_EINVAL, "n_incl_im must be finite and >= 0");
      if (v > 0) c->lossy = true;
    }
    if (c->lossy) {
      if (inc->shape) return set_err(c, GRT_EUNSUP, "absorbing inclusions must be disks");
      for (int64_t m = 0; m < M; ++m) {
        // the validated range of the complex-argument Bessel recurrence
        const double zr = wave->omega * inc->n_incl[m] * inc->radius[m];
        const double zi = wave->omega * inc->n_incl_im[m] * inc->radius[m];
        if (zi > 2.0 || std::hypot(zr, zi) > 40.0)
          return set_err(c, GRT_EUNSUP, "absorbing disk " + std::to_string(m) +
                                            ": Im(k_p R) > 2 or |k_p R| > 40");
      }
      c->hn_im.assign(inc->n_incl_im, inc->n_incl_im + M);
    }
  }
  if (inc->shape && M > 0) {
    // non-circular inclusions (eq. par1): a1 > 0, |a2| < a1, a3 a positive integer,
    // radius the enclosing circle a1 + |a2|
    if (R > 1) return set_err(c, GRT_EUNSUP, "non-circular inclusions with several angles");
    if (wave->P > 20) return set_err(c, GRT_EUNSUP, "non-circular inclusions need P <= 20");
    const int nodes = inc->shape_nodes > 0 ? inc->shape_nodes : 64;
    if (nodes < 16 || nodes > 512 || (nodes & 1))
      return set_err(c, GRT_EINVAL, "shape_nodes must be even, in [16, 512]");
    c->hshape.assign(inc->shape, inc->shape + 4 * M);
    c->shape_nodes = nodes;
    for (int64_t m = 0; m < M; ++m) {
      const double a1 = c->hshape[4 * m], a2 = c->hshape[4 * m + 1];
      const double a3 = c->hshape[4 * m + 2], rot = c->hshape[4 * m + 3];
      if (!std::isfinite(a1) || !std::isfinite(a2) || !std::isfinite(rot) || !(a1 > 0) ||
          !(std::fabs(a2) < a1) || !(a3 >= 1 && a3 <= 64 && a3 == std::floor(a3)))
        return set_err(c, GRT_EINVAL, "bad shape of inclusion " + std::to_string(m));
      const double rr = a1 + std::fabs(a2);
      if (!(std::fabs(inc->radius[m] - rr) <= 1e-12 * rr))
        return set_err(c, GRT_EINVAL, "radius of inclusion " + std::to_string(m) +
                                          " must be its enclosing circle a1 + |a2|");
    }
  }
  for (int64_t m = 0; m < M; ++m) {
    if (!std::isfinite(c->hx[m]) || !std::isfinite(c->hy[m]) || !finite_pos(c->hr[m]) ||
        !finite_pos(c->hn[m]))
      return set_err(c, GRT_EINVAL, "non-finite or non-positive inclusion data");
    if (F == 0 && std::fabs(c->hy[m]) + c->hr[m] >= L.h)
      return set_err(c, GRT_EGEOM, "inclusion " + std::to_string(m) + " touches an interface");
    if (F > 0) {
      // the centre between the graphs, and no graph point within the radius (sampled
      // over the disk's x-range at spacing radius / 256)
      const double xc = c->hx[m], yc = c->hy[m], r = c->hr[m];
      bool hit = !(yc < iface_height(iface.data(), F, 0, L.h, L.d, xc, 0) &&
                   yc > iface_height(iface.data(), F, 1, L.h, L.d, xc, 0));
      for (int j = 0; j < 2 && !hit; ++j)
        for (int i = -256; i <= 256 && !hit; ++i) {
          const double x = xc + r * i / 256.0;
          const double dy = iface_height(iface.data(), F, j, L.h, L.d, x, 0) - yc;
          hit = (x - xc) * (x - xc) + dy * dy <= r * r;
        }
      if (hit)
        return set_err(c, GRT_EGEOM, "inclusion " + std::to_string(m) + " touches an interface");
    }
    if (std::fabs(c->hx[m]) > 0.5 * L.d)
      return set_err(c, GRT_EGEOM, "inclusion " + std::to_string(m) + " lies outside the cell |x| <= d/2");
  }
  // minimum-image overlap check on a cell grid
  if (M > 1) {
    double rmax = *std::max_element(c->hr.begin(), c->hr.end());
    double cell = std::max(2.0 * rmax, 1e-12);
    int ncx = std::max(1, (int)(L.d / cell));
    int ncy = std::max(1, (int)(2 * L.h / cell));
    std::vector<std::vector<int>> grid((size_t)ncx * ncy);
    auto cidx = [&](double x, double y, int& gx, int& gy) {
      double xw = x - L.d * std::floor(x / L.d + 0.5);
      gx = std::min(ncx - 1, std::max(0, (int)((xw + 0.5 * L.d) / (L.d / ncx))));
      gy = std::min(ncy - 1, std::max(0, (int)((y + L.h) / (2 * L.h / ncy))));
    };
    for (int64_t m = 0; m < M; ++m) {
      int gx, gy;
      cidx(c->hx[m], c->hy[m], gx, gy);
      for (int ox = -1; ox <= 1; ++ox)
        for (int oy = -1; oy <= 1; ++oy) {
          int qx = ((gx + ox) % ncx + ncx) % ncx, qy = gy + oy;
          if (qy < 0 || qy >= ncy) continue;
          for (int o : grid[(size_t)qx * ncy + qy]) {
            double dx = c->hx[m] - c->hx[o];
            dx -= L.d * std::floor(dx / L.d + 0.5);
            double dy = c->hy[m] - c->hy[o];
            double rr = c->hr[m] + c->hr[o];
            if (dx * dx + dy * dy <= rr * rr)
              return set_err(c, GRT_EGEOM, "inclusions " + std::to_string(o) + " and " +
                                               std::to_string(m) + " overlap");
          }
        }
      grid[(size_t)gx * ncy + gy].push_back((int)m);
    }
  }
  c->lay = L;
  c->lay.iface = nullptr;  // the caller's array: the context keeps its own copy
  c->hiface = iface;
  c->inc = *wave;
  c->inc.phi = phi0;
  c->inc.n_rhs = 0;
  c->inc.phis = nullptr;
  c->M = M;
  c->P = wave->P;
  c->nb = 2 * wave->P + 1;
  c->n_beta = M * c->nb;
  // derived device geometry
  DevGeom& g = c->g;
  g = DevGeom{};
  g.d = L.d;
  g.h = L.h;
  g.y0 = L.y0;
  g.hs = L.d / L.N;
  for (int l = 0; l < 3; ++l) {
    g.k[l] = wave->omega * L.n_layer[l];
    g.k_im[l] = l == 2 ? wave->omega * L.n3_im : 0.0;
    g.Nw[l] = L.Nw[l];
    g.Q[l] = L.Q[l];
  }
  g.te = wave->polarization == GRT_TE ? 1 : 0;
  g.curved = F > 0 ? 1 : 0;
  for (int l = 0; l < 3; ++l) {
    const double eps = L.n_layer[l] * L.n_layer[l];
    g.pv[l] = g.te ? eps : 1.0;
    g.fl[l] = g.te ? 1.0 / eps : 1.0;
  }
  if (g.te && L.n3_im > 0) {  // eps_3 = (n_3 + i n3_im)^2 and its inverse
    const cd e3 = cd{L.n_layer[2], L.n3_im} * cd{L.n_layer[2], L.n3_im};
    const cd ie3 = cdiv(cd{1.0, 0.0}, e3);
    g.pv[2] = e3.r;
    g.pv_im[2] = e3.i;
    g.fl[2] = ie3.r;
    g.fl_im[2] = ie3.i;
  }
  g.kappa = g.k[0] * std::sin(phi0);
  g.alpha = cd{std::cos(g.kappa * L.d), std::sin(g.kappa * L.d)};
  g.alpha_inv = cd{g.alpha.r, -g.alpha.i};
  g.N = L.N;
  g.Nu = L.Nu;
  g.n_rb_lo = L.n_rb_lo;
  g.Nrb = L.Nrb;
  g.zeta_K = L.zeta_K;
  g.P = wave->P;
  g.M = (int)M;
  g.jcy[0] = 0.5 * (L.h + L.y0);
  g.jcy[1] = 0.0;
  g.jcy[2] = -0.5 * (L.h + L.y0);
  int rs[RB_COUNT] = {L.N, L.N, L.N, L.N, L.Nw[1], L.Nw[1], L.Nw[0], L.Nw[0],
                      L.Nw[2], L.Nw[2], L.Nu, L.Nu, L.Nu, L.Nu};
  g.row_off[0] = 0;
  for (int b = 0; b < RB_COUNT; ++b) g.row_off[b + 1] = g.row_off[b] + rs[b];
  int cs[CB_COUNT] = {L.N, L.N, L.N, L.N, 2 * L.Q[1] + 1, 2 * L.Q[0] + 1, 2 * L.Q[2] + 1,
                      L.Nrb, L.Nrb};
  g.col_off[0] = 0;
  for (int b = 0; b < CB_COUNT; ++b) g.col_off[b + 1] = g.col_off[b] + cs[b];
  g.n_rows = g.row_off[RB_COUNT];
  g.n_alpha = g.col_off[CB_COUNT];
  c->n_g = g.row_off[RB_W1V];
  c->n_b = g.col_off[CB_A1];
  // the other angles: contexts of their own on the same device and stream
  c->n_rhs = R;
  c->phis.clear();
  if (R > 1) c->phis.assign(wave->phis, wave->phis + R);
  destroy_rhs(c, (size_t)(R - 1));
  for (int64_t r = 1; r < R; ++r) {
    if ((size_t)r > c->rhs.size()) {
      grt_ctx* sub = nullptr;
      grt_status st = grt_create(&sub, c->device, c->stream);
      if (st != GRT_OK) return set_err(c, st, "creating the context of an angle failed");
      sub->want_table = c->want_table;
      sub->table_lanes = c->table_lanes;
      c->rhs.push_back(sub);
    }
    grt_incidence w1 = *wave;
    w1.phi = wave->phis[r];
    w1.n_rhs = 0;
    w1.phis = nullptr;
    grt_status st = grt_set_problem(c->rhs[(size_t)r - 1], lay, inc, &w1);
    if (st != GRT_OK) return set_err(c, st, std::string("angle ") + std::to_string(r) + ": " +
                                                c->rhs[(size_t)r - 1]->err);
  }
  c->have_problem = true;
  return GRT_OK;
}

static grt_status upload_inclusions(grt_ctx* c) {
  const int64_t M = c->M;
  if (M > 0) {
    std::vector<double> kp(M);
    for (int64_t m = 0; m < M; ++m) kp[m] = c->inc.omega * c->hn[m];
    GRT_HIP(c, hipMalloc(&c->d_cx, sizeof(double) * M));
    GRT_HIP(c, hipMalloc(&c->d_cy, sizeof(double) * M));
    GRT_HIP(c, hipMalloc(&c->d_rad, sizeof(double) * M));
    GRT_HIP(c, hipMalloc(&c->d_kp, sizeof(double) * M));
    GRT_HIP(c, hipMemcpy(c->d_cx, c->hx.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    GRT_HIP(c, hipMemcpy(c->d_cy, c->hy.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    GRT_HIP(c, hipMemcpy(c->d_rad, c->hr.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    GRT_HIP(c, hipMemcpy(c->d_kp, kp.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    if (c->lossy) {
      for (int64_t m = 0; m < M; ++m) kp[m] = c->inc.omega * c->hn_im[m];
      GRT_HIP(c, hipMalloc(&c->d_kp_im, sizeof(double) * M));
      GRT_HIP(c, hipMemcpy(c->d_kp_im, kp.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    }
  }
  return GRT_OK;
}

grt_status grt_build_translation(grt_ctx* c) {
  GRT_CHECK_CTX(c);
  if (!c->have_problem) return set_err(c, GRT_ESTATE, "set_problem first");
  GRT_HIP(c, hipSetDevice(c->device));
  if (c->built || c->trans_built) return GRT_OK;
  grt_status st = upload_inclusions(c);
  if (st == GRT_OK) st = setup_translation(c);
  if (st == GRT_OK) st = apply_alloc(c);
  if (st != GRT_OK) {
    free_all(c);
    return st;
  }
  c->trans_built = true;
  return GRT_OK;
}

grt_status grt_build(grt_ctx* c) {
  GRT_CHECK_CTX(c);
  if (!c->have_problem) return set_err(c, GRT_ESTATE, "set_problem first");
  GRT_HIP(c, hipSetDevice(c->device));
  if (c->built) return GRT_OK;
  if (c->trans_built) free_all(c);   // start again with the layered structure
  grt_status st = upload_inclusions(c);
  if (st != GRT_OK) return st;
  st = setup_build(c);
  if (st != GRT_OK) return st;
  st = apply_alloc(c);
  if (st != GRT_OK) return st;
  if (c->want_table) {
    st = table_set(c, true);
    if (st != GRT_OK) return st;
  }
  if (c->want_table32) {
    st = table32_set(c, true);
    if (st != GRT_OK) return st;
  }
  for (grt_ctx* sub : c->rhs) {
    st = grt_build(sub);
    if (st != GRT_OK) return set_err(c, st, "building an angle: " + sub->err);
  }
  c->built = true;
  return GRT_OK;
}

grt_status grt_set_table(grt_ctx* c, int mode) {
  GRT_CHECK_CTX(c);
  if (mode < 0 || mode > 2) return set_err(c, GRT_EINVAL, "table mode must be 0, 1 or 2");
  for (grt_ctx* sub : c->rhs) {
    grt_status st = grt_set_table(sub, mode);
    if (st != GRT_OK) return set_err(c, st, "angle: " + sub->err);
  }
  c->want_table = mode != 0;
  c->table_lanes = mode == 2 ? 2 : 1;
  if (!c->built) return GRT_OK;
  return table_set(c, c->want_table);
}

grt_status grt_set_table32(grt_ctx* c, int on) {
  GRT_CHECK_CTX(c);
  if (on != 0 && on != 1) return set_err(c, GRT_EINVAL, "on must be 0 or 1");
  if (c->have_problem && c->n_rhs > 1 && on)
    return set_err(c, GRT_EUNSUP, "with several angles the FP32 translation is the "
                                  "matrix-core block product (no table)");
  c->want_table32 = on != 0;
  if (!c->built) return GRT_OK;
  return table32_set(c, c->want_table32);
}

grt_status grt_table_bytes(const grt_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return GRT_EINVAL;
  if (!c->have_problem) return GRT_ESTATE;
  *bytes = (int64_t)table_bytes(c);
  return GRT_OK;
}

grt_status grt_query(const grt_ctx* c, grt_sizes* out) {
  if (!c || !out) return GRT_EINVAL;
  if (!c->have_problem) return GRT_ESTATE;
  out->M = c->M;
  out->P = c->P;
  out->n_beta = c->n_beta;
  out->n_rows = c->g.n_rows;
  out->n_alpha = c->g.n_alpha;
  out->rank = c->built ? c->rank : 0;
  out->Nrb = c->g.Nrb;
  out->m2l_chunks = (c->built || c->trans_built) ? c->m2l_nchunks : 0;
  out->m2l_split = !c->built ? 0 : c->d_table ? c->table_lanes : c->m2l_split;
  out->cx_chunks = c->built ? c->c_nchunks : 0;
  out->bx_chunks = c->built ? c->b_nchunks : 0;
  out->n_rhs = c->n_rhs;
  return GRT_OK;
}

static grt_status check_built(grt_ctx* c) {
  if (!c->built)
    return set_err(c, GRT_ESTATE, c->trans_built ? "translation-only build: grt_build first"
                                                 : "build first");
  GRT_HIP(c, hipSetDevice(c->device));
  return GRT_OK;
}

// Calls that need only the translation data (grt_build or grt_build_translation).
static grt_status check_translation(grt_ctx* c) {
  if (!c->built && !c->trans_built) return set_err(c, GRT_ESTATE, "build first");
  GRT_HIP(c, hipSetDevice(c->device));
  return GRT_OK;
}

namespace {
// out[m][l][n] = mie[m][l] if l == n, else 0
__global__ void mie_blocks_kernel(int64_t tot, int nb, const cd* mie, cd* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const int64_t m = e / ((int64_t)nb * nb);
  const int r = (int)(e - m * nb * nb);
  const int l = r / nb, n = r - l * nb;
  out[e] = l == n ? mie[m * nb + l] : cd{0.0, 0.0};
}
}  // namespace

grt_status grt_scattering_blocks(grt_ctx* c, void* out) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);
  if (st != GRT_OK) return st;
  if (!out) return set_err(c, GRT_EINVAL, "null output");
  const int nb = 2 * c->P + 1;
  const size_t n = (size_t)c->M * nb * nb;
  if (n == 0) return GRT_OK;
  cd* o = static_cast<cd*>(out);
  if (c->d_sblk) {
    GRT_HIP(c, hipMemcpyAsync(o, c->d_sblk, sizeof(cd) * n, hipMemcpyDeviceToDevice, c->stream));
  } else {
    // disks: the Mie diagonal
    const int64_t tot = (int64_t)n;
    mie_blocks_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, c->stream>>>(tot, nb, c->d_mie, o);
    GRT_HIP(c, hipGetLastError());
  }
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  return GRT_OK;
}


extern "C++" {
// Run fn(context of angle r, offset of its vectors) for every right-hand side.
template <typename F>
static grt_status for_each_rhs(grt_ctx* c, F fn) {
  for (int64_t r = 0; r < c->n_rhs; ++r) {
    grt_ctx* cr = rhs_ctx(c, r);
    grt_status st = fn(cr, r * c->n_beta);
    if (st != GRT_OK) return cr == c ? st : set_err(c, st, "angle " + std::to_string(r) + ": " + cr->err);
  }
  return GRT_OK;
}
}  // extern "C++"

// Phases alpha_r of every angle and the block buffers for them.
static grt_status block_ready(grt_ctx* c) {
  std::vector<cd> al((size_t)c->n_rhs);
  for (int64_t r = 0; r < c->n_rhs; ++r) al[(size_t)r] = rhs_ctx(c, r)->g.alpha;
  return block_prepare(c, (int)c->n_rhs, al.data());
}

// y_r = K_r x_r for every angle with the translation of all angles at once on the
// FP32 matrix cores; the layer correction of each angle in FP64.
static grt_status apply_K_block(grt_ctx* c, const cd* x, cd* y) {
  const int R = (int)c->n_rhs;
  grt_status st = block_ready(c);
  if (st != GRT_OK) return st;
  if (!c->d_blkw) GRT_HIP(c, hipMalloc(&c->d_blkw, sizeof(cd) * (size_t)c->n_beta * R));
  st = block_product(c, x, c->n_beta, c->d_dnorm, R, c->stream);
  if (st != GRT_OK) return st;
  st = for_each_rhs(c, [&](grt_ctx* cr, int64_t off) {
    return apply_lowrank_only(cr, x + off, c->d_blkw + off);
  });
  if (st != GRT_OK) return st;
  block_combine(c, x, c->d_blkw, R, y, c->stream);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

grt_status grt_apply(grt_ctx* c, const void* x, void* y, int precision) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (!x || !y || x == y) return set_err(c, GRT_EINVAL, "bad vectors");
  const cd* xc = static_cast<const cd*>(x);
  cd* yc = static_cast<cd*>(y);
  if (precision == GRT_FP64)
    return for_each_rhs(c, [&](grt_ctx* cr, int64_t off) { return apply_K(cr, xc + off, yc + off); });
  if (precision == GRT_FP32) {
    if (c->n_rhs > 1 && c->M > 0) return apply_K_block(c, xc, yc);
    return apply_K_mixed(c, xc, yc);
  }
  return set_err(c, GRT_EINVAL, "precision must be GRT_FP64 or GRT_FP32");
}

grt_status grt_apply_T(grt_ctx* c, const void* x, void* y) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);
  if (st != GRT_OK) return st;
  if (!c->built && c->n_rhs > 1)
    return set_err(c, GRT_ESTATE, "translation-only build with several angles: use grt_apply_ST_block");
  if (!x || !y || x == y) return set_err(c, GRT_EINVAL, "bad vectors");
  const cd* xc = static_cast<const cd*>(x);
  cd* yc = static_cast<cd*>(y);
  return for_each_rhs(c, [&](grt_ctx* cr, int64_t off) { return apply_T_only(cr, xc + off, yc + off); });
}

grt_status grt_apply_ST_block(grt_ctx* c, const void* x, void* y) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);
  if (st != GRT_OK) return st;
  if (!x || !y || x == y) return set_err(c, GRT_EINVAL, "bad vectors");
  if (c->M == 0) return GRT_OK;
  if (has_shapes(c))
    return set_err(c, GRT_EUNSUP, "the block translation takes disks (Mie diagonal) only");
  st = block_ready(c);
  if (st != GRT_OK) return st;
  st = block_product(c, static_cast<const cd*>(x), c->n_beta, c->d_dnorm, (int)c->n_rhs, c->stream);
  if (st != GRT_OK) return st;
  block_unpack(c, (int)c->n_rhs, static_cast<cd*>(y), c->stream);
  GRT_HIP(c, hipGetLastError());
  return GRT_OK;
}

grt_status grt_apply_lowrank(grt_ctx* c, const void* x, void* y) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (!x || !y || x == y) return set_err(c, GRT_EINVAL, "bad vectors");
  const cd* xc = static_cast<const cd*>(x);
  cd* yc = static_cast<cd*>(y);
  return for_each_rhs(c, [&](grt_ctx* cr, int64_t off) {
    return apply_lowrank_only(cr, xc + off, yc + off);
  });
}

grt_status grt_rhs(grt_ctx* c, void* b) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (!b) return set_err(c, GRT_EINVAL, "null vector");
  cd* bc = static_cast<cd*>(b);
  return for_each_rhs(c, [&](grt_ctx* cr, int64_t off) { return rhs_b(cr, bc + off); });
}

grt_status grt_set_overlap(grt_ctx* c, int on) {
  GRT_CHECK_CTX(c);
  if (on != 0 && on != 1) return set_err(c, GRT_EINVAL, "overlap must be 0 or 1");
  GRT_HIP(c, hipSetDevice(c->device));
  if (on && !c->stream2) {
    GRT_HIP(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
    GRT_HIP(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    GRT_HIP(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  c->overlap = on != 0;
  graph_reset(c);
  for (grt_ctx* sub : c->rhs) {
    grt_status st = grt_set_overlap(sub, on);
    if (st != GRT_OK) return set_err(c, st, "angle: " + sub->err);
  }
  return GRT_OK;
}

grt_status grt_set_fmm(grt_ctx* c, int enable, int p_cell, int per_cell, int* info) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);
  if (st != GRT_OK) return st;
  if (enable != 0 && enable != 1) return set_err(c, GRT_EINVAL, "enable must be 0 or 1");
  if (p_cell < 0 || per_cell < 0) return set_err(c, GRT_EINVAL, "p_cell, per_cell must be >= 0");
  if (enable && c->n_rhs > 1)
    return set_err(c, GRT_EUNSUP, "the cell translation takes one angle");
  GRT_HIP(c, hipSetDevice(c->device));
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  graph_reset(c);
  ++c->gen;
  if (!enable) {
    fmm_release(c);
  } else {
    st = fmm_setup(c, p_cell, per_cell);
    if (st != GRT_OK) return st;
  }
  if (info) {
    info[0] = c->fmm_on ? c->fmm_nx : 0;
    info[1] = c->fmm_on ? c->fmm_ny : 0;
    info[2] = c->fmm_on ? c->fmm_p : 0;
  }
  return GRT_OK;
}

grt_status grt_set_launch(grt_ctx* c, int m2l_chunks, int m2l_split) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);
  if (st != GRT_OK) return st;
  if (m2l_split != 1 && m2l_split != 2) return set_err(c, GRT_EINVAL, "split must be 1 or 2");
  if (c->M == 0) return GRT_OK;
  if (m2l_chunks < 1 || m2l_chunks > c->m2l_nchunks_cap || m2l_chunks > c->M)
    return set_err(c, GRT_EINVAL, "chunk count must be in [1, " +
                                      std::to_string(std::min<int64_t>(c->m2l_nchunks_cap, c->M)) + "]");
  const int64_t ch = (c->M + m2l_chunks - 1) / m2l_chunks;
  c->m2l_chunk = (int)ch;
  c->m2l_nchunks = (int)((c->M + ch - 1) / ch);
  if (c->d_table)
    c->table_lanes = m2l_split;
  else
    c->m2l_split = m2l_split;
  graph_reset(c);
  ++c->gen;   // a batch made earlier holds the old launch shape
  for (grt_ctx* sub : c->rhs) {
    if (!sub->built) continue;
    grt_status st2 = grt_set_launch(sub, m2l_chunks, m2l_split);
    if (st2 != GRT_OK) return set_err(c, st2, "angle: " + sub->err);
  }
  return GRT_OK;
}

grt_status grt_autotune(grt_ctx* c, int cap, int* n, int* chunks, int* splits, double* ms) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (cap < 0 || (cap > 0 && (!chunks || !ms))) return set_err(c, GRT_EINVAL, "bad arrays");
  st = autotune_m2l(c, cap, n, chunks, splits, ms);
  if (st != GRT_OK) return st;
  st = autotune_coupling(c);
  if (st != GRT_OK) return st;
  // the other angles share the geometry: they take the same launch shapes
  for (grt_ctx* sub : c->rhs) {
    sub->m2l_chunk = c->m2l_chunk;
    sub->m2l_nchunks = c->m2l_nchunks;
    sub->m2l_split = c->m2l_split;
    sub->table_lanes = c->table_lanes;
    sub->c_chunk = c->c_chunk;
    sub->c_nchunks = c->c_nchunks;
    sub->b_chunk = c->b_chunk;
    sub->b_nchunks = c->b_nchunks;
    graph_reset(sub);
    ++sub->gen;
  }
  ++c->gen;
  return GRT_OK;
}

grt_status grt_incident(grt_ctx* c, void* a) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (!a) return set_err(c, GRT_EINVAL, "null vector");
  cd* ac = static_cast<cd*>(a);
  return for_each_rhs(c, [&](grt_ctx* cr, int64_t off) { return incident_alpha(cr, ac + off); });
}

// Every angle of a context with several right-hand sides: one lockstep batch over the
// angles' contexts (FP32 precision translates all angles at once on the matrix cores).
static grt_status solve_block(grt_ctx* c, const grt_solve_opts* o, cd* beta,
                              grt_solve_stats* stats) {
  const int64_t R = c->n_rhs;
  std::vector<grt_ctx*> list((size_t)R);
  std::vector<void*> ptrs((size_t)R);
  for (int64_t r = 0; r < R; ++r) {
    list[(size_t)r] = rhs_ctx(c, r);
    ptrs[(size_t)r] = beta + r * c->n_beta;
  }
  std::vector<grt_solve_stats> tmp((size_t)R);
  grt_solve_stats* sp = stats ? stats : tmp.data();
  grt_status st = GRT_OK;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (!c->rhs_batch) {
      st = batch_create_internal(&c->rhs_batch, R, list.data(), c->stream);
      if (st != GRT_OK) return set_err(c, st, "batch of the angles could not be made");
      st = batch_set_block(c->rhs_batch, c);
      if (st != GRT_OK) return set_err(c, st, grt_batch_error_message(c->rhs_batch));
    }
    if (o->precision != GRT_FP64) {
      st = block_ready(c);
      if (st != GRT_OK) return st;
    }
    st = grt_batch_solve(c->rhs_batch, o, ptrs.data(), sp);
    if (st == GRT_ESTATE && attempt == 0) {   // an angle changed since the batch was made
      grt_batch_destroy(c->rhs_batch);
      c->rhs_batch = nullptr;
      continue;
    }
    break;
  }
  if (st != GRT_OK) set_err(c, st, grt_batch_error_message(c->rhs_batch));
  return st;
}

grt_status grt_solve(grt_ctx* c, const grt_solve_opts* o, void* beta, grt_solve_stats* stats) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  if (!o || !beta) return set_err(c, GRT_EINVAL, "null argument");
  if (!(o->tol > 0 && o->tol < 1)) return set_err(c, GRT_EINVAL, "tol must be in (0, 1)");
  if (o->precision != GRT_FP64 && o->precision != GRT_FP32 && o->precision != GRT_FP32_RELAXED)
    return set_err(c, GRT_EINVAL, "precision must be GRT_FP64, GRT_FP32 or GRT_FP32_RELAXED");
  if (c->fmm_on && o->precision != GRT_FP64)
    return set_err(c, GRT_EUNSUP, "the cell translation is FP64 only");
  grt_solve_stats tmp{};
  grt_solve_stats* sp = stats ? stats : &tmp;
  if (c->M == 0) {
    for (int64_t r = 0; r < (stats ? c->n_rhs : 1); ++r) sp[r] = grt_solve_stats{};
    return GRT_OK;
  }
  if (c->n_rhs > 1) return solve_block(c, o, static_cast<cd*>(beta), stats);
  return gmres_solve(c, o, static_cast<cd*>(beta), sp);
}

namespace {
// R_n, T_n for the propagating orders and the flux error |sum R + sum T - 1|.
__global__ void bragg_finish_kernel(DevGeom g, double k1cos, const cd* cdv, double* R, double* T,
                                    double* flux) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  const bool lossy3 = g.k_im[2] != 0.0;
  for (int i = 0; i < g.Nrb; ++i) {
    double kapn = g.kappa + 2.0 * M_PI * (g.n_rb_lo + i) / g.d;
    double v1 = g.k[0] * g.k[0] - kapn * kapn;
    double v3 = g.k[2] * g.k[2] - kapn * kapn;
    double r = v1 > 0 ? sqrt(v1) * cabs2(cdv[i]) / k1cos : 0.0;
    // TE: the flux of a wave is (k_y / eps) |amplitude|^2.  Absorbing substrate: every
    // order carries Re(k_3n) |d_n|^2 across Gamma_d.
    double t;
    if (lossy3) {
      const cd k3{g.k[2], g.k_im[2]};
      const cd k3n = csqrt_principal(k3 * k3 - cd{kapn * kapn, 0.0});
      // TE: Re(k_3n / eps_3) eps_1
      const double ky = g.te ? g.pv[0] * (k3n * cd{g.fl[2], g.fl_im[2]}).r : k3n.r;
      t = ky * cabs2(cdv[g.Nrb + i]) / k1cos;
    } else {
      t = v3 > 0 ? (g.pv[0] / g.pv[2]) * sqrt(v3) * cabs2(cdv[g.Nrb + i]) / k1cos : 0.0;
    }
    R[i] = r;
    T[i] = t;
    s += r + t;
  }
  // absorbing substrate: it also absorbs between Gamma_2 and Gamma_d, so R + T + A
  // is no energy balance
  *flux = lossy3 ? __builtin_nan("") : fabs(s - 1.0);
}
}  // namespace

// Fraction of the incident flux absorbed by the disks (see grating.h): from beta and
// the Mie diagonal on the host.
static grt_status absorbed_fraction(grt_ctx* c, const cd* beta, double* out) {
  *out = 0.0;
  if (!c->lossy || c->M == 0) return GRT_OK;
  std::vector<cd> b(c->n_beta), s(c->n_beta);
  GRT_HIP(c, hipMemcpyAsync(b.data(), beta, sizeof(cd) * c->n_beta, hipMemcpyDeviceToHost,
                            c->stream));
  GRT_HIP(c, hipMemcpyAsync(s.data(), c->d_mie, sizeof(cd) * c->n_beta, hipMemcpyDeviceToHost,
                            c->stream));
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  double acc = 0.0;
  for (int64_t i = 0; i < c->n_beta; ++i) {
    const double s2 = s[i].r * s[i].r + s[i].i * s[i].i;
    if (s2 > 0) acc += (b[i].r * b[i].r + b[i].i * b[i].i) * (s2 + s[i].r) / s2;
  }
  const double w = c->g.te ? c->g.pv[0] / c->g.pv[1] : 1.0;  // eps_1 / eps_2
  *out = -4.0 * w * acc / (c->g.d * c->g.k[0] * std::cos(c->inc.phi));
  return GRT_OK;
}

grt_status grt_bragg(grt_ctx* c0, int64_t rhs, const void* beta, int64_t cap, int* orders,
                     double* cc, double* dd, double* R, double* T, double* flux_err,
                     double* absorbed) {
  GRT_CHECK_CTX(c0);
  grt_status st = check_built(c0);
  if (st != GRT_OK) return st;
  if (rhs < 0 || rhs >= c0->n_rhs) return set_err(c0, GRT_EINVAL, "rhs out of range");
  grt_ctx* c = rhs_ctx(c0, rhs);
  if (c != c0) {
    st = grt_bragg(c, 0, beta, cap, orders, cc, dd, R, T, flux_err, absorbed);
    return st == GRT_OK ? st : set_err(c0, st, c->err);
  }
  const int Nrb = c->g.Nrb;
  if (cap < Nrb || !orders || !cc || !dd || !R || !T || !flux_err)
    return set_err(c, GRT_EINVAL, "output arrays too small or null");
  if (c->M > 0 && !beta) return set_err(c, GRT_EINVAL, "null beta");
  cd* dcd = nullptr;
  double* dr = nullptr;
  GRT_HIP(c, hipMalloc(&dcd, sizeof(cd) * 2 * Nrb));
  GRT_HIP(c, hipMalloc(&dr, sizeof(double) * (2 * Nrb + 1)));
  st = bragg_alpha(c, static_cast<const cd*>(beta), dcd);
  if (st == GRT_OK) {
    bragg_finish_kernel<<<1, 64, 0, c->stream>>>(c->g, c->g.k[0] * std::cos(c->inc.phi), dcd, dr,
                                                 dr + Nrb, dr + 2 * Nrb);
    std::vector<cd> hcd(2 * Nrb);
    std::vector<double> hr(2 * Nrb + 1);
    hipError_t e1 = hipMemcpyAsync(hcd.data(), dcd, sizeof(cd) * 2 * Nrb, hipMemcpyDeviceToHost, c->stream);
    hipError_t e2 = hipMemcpyAsync(hr.data(), dr, sizeof(double) * (2 * Nrb + 1), hipMemcpyDeviceToHost, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      st = set_err(c, GRT_EHIP, "bragg copy failed");
    } else {
      for (int i = 0; i < Nrb; ++i) {
        orders[i] = c->g.n_rb_lo + i;
        cc[2 * i] = hcd[i].r;
        cc[2 * i + 1] = hcd[i].i;
        dd[2 * i] = hcd[Nrb + i].r;
        dd[2 * i + 1] = hcd[Nrb + i].i;
        R[i] = hr[i];
        T[i] = hr[Nrb + i];
      }
      *flux_err = hr[2 * Nrb];
      double ab = 0.0;
      st = absorbed_fraction(c, static_cast<const cd*>(beta), &ab);
      if (st == GRT_OK && c->lossy && c->g.k_im[2] == 0.0) {  // else no balance (NaN)
        double sum = ab - 1.0;
        for (int i = 0; i < Nrb; ++i) sum += R[i] + T[i];
        *flux_err = std::fabs(sum);
      }
      if (absorbed) *absorbed = ab;
    }
  }
  hipFree(dcd);
  hipFree(dr);
  return st;
}

grt_status grt_get_A(grt_ctx* c, double* A_host, double* colscale_host) {
  GRT_CHECK_CTX(c);
  grt_status st = check_built(c);
  if (st != GRT_OK) return st;
  size_t nA = (size_t)c->g.n_rows * c->g.n_alpha;
  if (A_host) GRT_HIP(c, hipMemcpy(A_host, c->d_A, sizeof(cd) * nA, hipMemcpyDeviceToHost));
  if (colscale_host)
    GRT_HIP(c, hipMemcpy(colscale_host, c->d_colscale, sizeof(double) * c->g.n_alpha,
                         hipMemcpyDeviceToHost));
  return GRT_OK;
}

grt_status grt_profile_enable(grt_ctx* c, int enable) {
  GRT_CHECK_CTX(c);
  c->prof = enable != 0;
  return GRT_OK;
}

grt_status grt_profile_read(grt_ctx* c, double* m2l_ms_total, int64_t* m2l_launches) {
  GRT_CHECK_CTX(c);
  if (!m2l_ms_total || !m2l_launches) return set_err(c, GRT_EINVAL, "null output");
  GRT_HIP(c, hipSetDevice(c->device));
  GRT_HIP(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
    float ms = 0.0f;
    GRT_HIP(c, hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]));
    c->prof_ms += ms;
    c->prof_count += 1;
  }
  c->prof_used = 0;
  *m2l_ms_total = c->prof_ms;
  *m2l_launches = c->prof_count;
  c->prof_ms = 0.0;
  c->prof_count = 0;
  return GRT_OK;
}

grt_status grt_get_mie(grt_ctx* c, double* s_host) {
  GRT_CHECK_CTX(c);
  grt_status st = check_translation(c);  // the Mie diagonal is part of the translation build
  if (st != GRT_OK) return st;
  if (!s_host) return set_err(c, GRT_EINVAL, "null buffer");
  if (c->M > 0)
    GRT_HIP(c, hipMemcpy(s_host, c->d_mie, sizeof(cd) * c->n_beta, hipMemcpyDeviceToHost));
  return GRT_OK;
}

}  // extern "C"
