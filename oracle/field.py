"""The scattered and total field at arbitrary points, from the representation (oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 3 (eqs. repre1-repre3) and sec. 5 (eq. repre3_mod): in each truncated
layer the field is a sum over the near copies l = -1, 0, 1 (phased by alpha^l) of
single- and double-layer potentials on the interfaces it touches, plus a J
expansion about the layer's centre; the middle layer adds the outgoing multipoles
of every inclusion and of its two near copies (the far copies enter through the
middle J expansion).  The densities on both sides of an interface are the same
(sigma_i, mu_i), with the k of the layer evaluated:

  u_1 = S_{k1}[Gamma_1] sigma_1 + D_{k1}[Gamma_1] mu_1 + sum_q a1_q J_q(k1 |x - c1|) e^{iq theta}
  u_2 = S_{k2}[Gamma_1] sigma_1 + D_{k2}[Gamma_1] mu_1 + S_{k2}[Gamma_2] sigma_2 + D_{k2}[Gamma_2] mu_2
        + sum_q a2_q J_q(k2 |x - c2|) e^{iq theta}
        + sum_{m,l} alpha^l sum_n beta_m[n] H_n(k2 |x - c_m - l d e_x|) e^{in theta}
  u_3 = S_{k3}[Gamma_2] sigma_2 + D_{k3}[Gamma_2] mu_2 + sum_q a3_q J_q(k3 |x - c3|) e^{iq theta}

(S: kernel (i/4) H_0(k r); D: its derivative along the source normal +y), and
above Gamma_u / below Gamma_d the Rayleigh-Bloch expansions of eqs. rad1/rad2:
  u_1 = sum_n c_n e^{i kappa_n x + i k_{1,n} (y - y0)},  u_3 = sum_n d_n e^{i kappa_n x - i k_{3,n} (y + y0)}.
The total field in the top layer adds the incident plane wave.

Off-node evaluation.  The discretized layer potentials are trapezoid sums over the
interface nodes of the three copies (the field the method solves for).  Near a
line that sum is inaccurate, so inside a smooth window around the target it is
replaced by the integral of the densities' trigonometric interpolant (sigma
e^{-i kappa x} is periodic) on a fine grid, exponentially accurate for targets a
few fine spacings from the line.  Limits on an interface are taken from each side
by polynomial extrapolation in the distance (limit_on_line).  This evaluation
shares no quadrature with the assembly of A: no kernel splitting and no zeta
correction, and the jump relations are not imposed but come out of the near-line
sums.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .common import outgoing, incoming, grad_wave


def trig_interp(G, vals, xs):
    """Quasi-periodic trigonometric interpolant of node values at the points xs."""
    N = len(vals)
    w = np.asarray(vals) * np.exp(-1j * G.kappa * G.xg)
    m = np.arange(-(N // 2), N - N // 2)
    E = np.exp(-2j * np.pi * np.outer(m, G.xg) / G.d)
    coef = E @ w / N
    if N % 2 == 0:
        # split the Nyquist mode between -N/2 and +N/2: on the cell-centred nodes
        # e^{i pi N x / d} = -e^{-i pi N x / d}, so the halves take opposite signs
        # (a sine mode, matching the node values)
        c0 = coef[0] / 2
        coef = np.concatenate([[c0], coef[1:], [-c0]])
        m = np.concatenate([m, [N // 2]])
    ph = np.exp(2j * np.pi * np.outer(np.asarray(xs, float), m) / G.d)
    return (ph @ coef) * np.exp(1j * G.kappa * np.asarray(xs, float))


def _kernels(k, Rx, Ry):
    """Single layer (i/4) H0(k r), its source-normal (+y) derivative and their
    target gradients, R = target - source: (g, g_x, g_y, dd, dd_x, dd_y)."""
    r = np.hypot(Rx, Ry)
    H0 = sp.hankel1(0, k * r)
    H1 = sp.hankel1(1, k * r)
    # grad_t (i/4) H0(kr) = -(i k / 4) H1 R / r
    g = 0.25j * H0
    gx = -0.25j * k * H1 * Rx / r
    gy = -0.25j * k * H1 * Ry / r
    # d/dy_s (i/4) H0(k|t - s|) = (i k / 4) f(r) Ry with f = H1 / r, f' = k H0 / r - 2 H1 / r^2
    f = H1 / r
    fp = k * H0 / r - 2 * H1 / r ** 2
    dd = 0.25j * k * f * Ry
    ddx = 0.25j * k * fp * (Rx / r) * Ry
    ddy = 0.25j * k * (fp * (Ry / r) * Ry + f)
    return g, gx, gy, dd, ddx, ddy


def _window(s, w):
    return np.exp(-(s / w) ** 8)


def _line_field(G, k, ys, sig, mu, tx, ty, n_fine, width=0.12):
    """(u, du/dx, du/dy) of S_k sigma + D_k mu from the line y = ys (three copies).

    The discretized representation is the trapezoid sum over the N nodes of each
    copy: that is the field the method solves for (its quadrature error at the ends
    of the three-copy segment is smooth in the unit cell and taken up by the J
    expansion).  Close to the line that sum loses accuracy, so the part of it inside
    a smooth window chi(x_node - x_target) of half-width about 1.5 width is replaced
    by the integral of the interpolated densities against the same window on a fine
    grid; for targets more than six node spacings from the line the two agree to
    rounding and the node sum is kept.
    """
    tx = np.asarray(tx, float)[:, None]
    ty = np.asarray(ty, float)[:, None]
    w = width * G.d
    u = np.zeros(tx.shape[0], complex)
    ux = np.zeros_like(u)
    uy = np.zeros_like(u)
    # targets within six node spacings of the line get the windowed fine integral;
    # farther, the node sum is exact to rounding (error ~ exp(-2 pi dist / h))
    near = np.abs(ty - ys) <= 6.0 * G.hs
    # discrete sum over the nodes of the three copies, outside the window
    for l in (-1, 0, 1):
        a = G.alpha ** l
        xs = G.xg[None, :] + l * G.d
        keep = 1.0 - near * _window(xs - tx, w)
        g, gx, gy, dd, ddx, ddy = _kernels(k, tx - xs, ty - ys)
        sl = a * G.hs * keep
        u += (sl * g) @ sig + (sl * dd) @ mu
        ux += (sl * gx) @ sig + (sl * ddx) @ mu
        uy += (sl * gy) @ sig + (sl * ddy) @ mu
    # fine-grid integral inside the window (the interpolants carry the Bloch phase)
    hf = G.d / n_fine
    xf = -1.5 * G.d + (np.arange(3 * n_fine) + 0.5) * hf
    sf = trig_interp(G, sig, xf)
    mf = trig_interp(G, mu, xf)
    for i in range(tx.shape[0]):
        if not near[i, 0]:
            continue
        sel = np.abs(xf - tx[i, 0]) < 2.0 * w
        xs = xf[sel]
        wt = hf * _window(xs - tx[i, 0], w)
        g, gx, gy, dd, ddx, ddy = _kernels(k, tx[i, 0] - xs, ty[i, 0] - ys)
        u[i] += (wt * g) @ sf[sel] + (wt * dd) @ mf[sel]
        ux[i] += (wt * gx) @ sf[sel] + (wt * ddx) @ mf[sel]
        uy[i] += (wt * gy) @ sf[sel] + (wt * ddy) @ mf[sel]
    return u, ux, uy


def _jexp(G, layer, coef, tx, ty):
    Q = G.Q[layer]
    k = G.kl[layer]
    cx, cy = G.jc[layer]
    q = np.arange(-Q, Q + 1)[None, :]
    vx = (np.asarray(tx, float) - cx)[:, None]
    vy = (np.asarray(ty, float) - cy)[:, None]
    u = incoming(q, k, vx, vy) @ coef
    gx, gy = grad_wave(incoming, q, k, vx, vy)
    return u, gx @ coef, gy @ coef


def _inclusions(G, beta, tx, ty, skip=None):
    """Outgoing multipoles of every inclusion and its near copies (skip: (m, l) left out)."""
    P = G.P
    n = np.arange(-P, P + 1)[None, :]
    b = np.asarray(beta).reshape(G.M, 2 * P + 1)
    tx = np.asarray(tx, float)
    ty = np.asarray(ty, float)
    u = np.zeros(len(tx), complex)
    ux = np.zeros_like(u)
    uy = np.zeros_like(u)
    for m in range(G.M):
        for l in (-1, 0, 1):
            if skip is not None and (m, l) == skip:
                continue
            a = G.alpha ** l
            vx = (tx - G.cx[m] - l * G.d)[:, None]
            vy = (ty - G.cy[m])[:, None]
            u += a * (outgoing(n, G.k2, vx, vy) @ b[m])
            gx, gy = grad_wave(outgoing, n, G.k2, vx, vy)
            ux += a * (gx @ b[m])
            uy += a * (gy @ b[m])
    return u, ux, uy


def interior_coefficients(red, beta):
    """gamma_m[n] of the field inside disk m, sum_n gamma_n J_n(k_p r) e^{in theta}
    (sec. 4.1): continuity at r = R with the exterior sum_n (a_n J_n(k2 r) + beta_n
    H_n(k2 r)) e^{in theta}, where a = T beta + B_phys A^+ (f - C beta) is the field
    arriving at the disk (sec. 5)."""
    G = red.G
    P = G.P
    n = np.arange(-P, P + 1)[None, :]
    a = red.T_apply(beta) - red.lowrank_apply(beta) + red.B @ red.pinv.apply(red.f)
    a = a.reshape(G.M, 2 * P + 1)
    b = np.asarray(beta).reshape(G.M, 2 * P + 1)
    R = G.rad[:, None]
    ext = a * sp.jv(n, G.k2 * R) + b * sp.hankel1(n, G.k2 * R)
    return ext / sp.jv(n, G.kp[:, None] * R)


class Field:
    """Field of one solved problem: beta (inclusions) and alpha = A^+ (f - C beta)."""

    def __init__(self, red, beta, n_fine=16384):
        G = self.G = red.G
        if G.te:
            raise NotImplementedError("field evaluation is written for TM")
        if G.curved:
            raise NotImplementedError("field evaluation is written for flat interfaces")
        self.beta = np.zeros(0) if G.M == 0 else np.asarray(beta)
        # interior expansions exist for disks only; for the non-circular inclusions the
        # field is available outside their enclosing circles
        self.gamma = (interior_coefficients(red, self.beta)
                      if G.M and getattr(G.pb, "shape", None) is None else None)
        al = red.alpha_vec(self.beta)
        c = G.col
        self.mu1, self.sig1 = al[c["mu1"]], al[c["sig1"]]
        self.mu2, self.sig2 = al[c["mu2"]], al[c["sig2"]]
        self.a = (al[c["a1"]], al[c["a2"]], al[c["a3"]])
        self.c, self.d = al[c["c"]], al[c["d"]]
        self.n_fine = n_fine

    def layer(self, j, tx, ty, total=True, skip=None):
        """(u, u_x, u_y) of layer j's representation (0 top, 1 middle, 2 bottom) at
        the points (tx, ty); total adds the incident wave in the top layer; skip
        leaves one inclusion copy (m, l) out of the middle layer's sum."""
        G = self.G
        tx = np.atleast_1d(np.asarray(tx, float))
        ty = np.atleast_1d(np.asarray(ty, float))
        k = G.kl[j]
        parts = [_jexp(G, j, self.a[j], tx, ty)]
        if j in (0, 1):
            parts.append(_line_field(G, k, G.h, self.sig1, self.mu1, tx, ty, self.n_fine))
        if j in (1, 2):
            parts.append(_line_field(G, k, -G.h, self.sig2, self.mu2, tx, ty, self.n_fine))
        if j == 1 and G.M:
            parts.append(_inclusions(G, self.beta, tx, ty, skip))
        u = sum(p[0] for p in parts)
        ux = sum(p[1] for p in parts)
        uy = sum(p[2] for p in parts)
        if j == 0 and total:
            ui = G.u_inc(tx, ty)
            u = u + ui
            ux = ux + 1j * G.kappa * ui
            uy = uy - 1j * G.k1 * G.cosphi * ui
        return u, ux, uy

    def rayleigh(self, top, tx, ty):
        """(u, u_x, u_y) of the Rayleigh-Bloch expansion above y0 (top) or below -y0."""
        G = self.G
        tx = np.atleast_1d(np.asarray(tx, float))[:, None]
        ty = np.atleast_1d(np.asarray(ty, float))[:, None]
        if top:
            kn, coef, yy = G.k1n, self.c, ty - G.y0
        else:
            kn, coef, yy = -G.k3n, self.d, ty + G.y0
        E = np.exp(1j * (G.kapn[None, :] * tx + kn[None, :] * yy))
        return E @ coef, (1j * G.kapn[None, :] * E) @ coef, (1j * kn[None, :] * E) @ coef

    def inside(self, tx, ty):
        """(inside, value): which points lie in a disk or one of its near copies
        (x_m + l d, l = -1, 0, 1), and the interior field there (the copy's field is
        alpha^l times the disk's, by quasi-periodicity)."""
        G = self.G
        tx = np.atleast_1d(np.asarray(tx, float))
        ty = np.atleast_1d(np.asarray(ty, float))
        ins = np.zeros(len(tx), bool)
        val = np.zeros(len(tx), complex)
        n = np.arange(-G.P, G.P + 1)[None, :]
        for m in range(G.M):
            for l in (-1, 0, 1):
                vx = tx - G.cx[m] - l * G.d
                vy = ty - G.cy[m]
                sel = (np.hypot(vx, vy) < G.rad[m]) & ~ins
                if np.any(sel):
                    if self.gamma is None:
                        raise NotImplementedError("field inside the enclosing circle of a "
                                                  "non-circular inclusion")
                    J = incoming(n, G.kp[m], vx[sel][:, None], vy[sel][:, None])
                    val[sel] = G.alpha ** l * (J @ self.gamma[m])
                    ins |= sel
        return ins, val

    def total(self, tx, ty):
        """Total field (value only) at points of any layer, inclusions included.  The
        representation holds in the unit cell |x| <= d/2; elsewhere the field follows
        from quasi-periodicity, u(x + l d) = alpha^l u(x) (sec. 2, eq. bound2)."""
        G = self.G
        tx = np.atleast_1d(np.asarray(tx, float))
        ty = np.atleast_1d(np.asarray(ty, float))
        cell = np.floor(tx / G.d + 0.5)
        if np.any(cell != 0):
            return G.alpha ** cell * self.total(tx - cell * G.d, ty)
        out = np.zeros(len(tx), complex)
        if G.M:
            ins, val = self.inside(tx, ty)
            out[ins] = val[ins]
            if np.all(ins):
                return out
            rest = ~ins
            out[rest] = self._outside(tx[rest], ty[rest])
            return out
        return self._outside(tx, ty)

    def _outside(self, tx, ty):
        G = self.G
        out = np.zeros(len(tx), complex)
        for sel, fn in ((ty > G.y0, lambda x, y: self.rayleigh(True, x, y)[0]
                         + G.u_inc(x, y)),
                        ((ty <= G.y0) & (ty > G.h), lambda x, y: self.layer(0, x, y)[0]),
                        ((ty <= G.h) & (ty >= -G.h), lambda x, y: self.layer(1, x, y)[0]),
                        ((ty < -G.h) & (ty >= -G.y0), lambda x, y: self.layer(2, x, y)[0]),
                        (ty < -G.y0, lambda x, y: self.rayleigh(False, x, y)[0])):
            if np.any(sel):
                out[sel] = fn(tx[sel], ty[sel])
        return out

    def limit_on_line(self, j, x0, y_line, side, delta=5e-4, npts=8):
        """Limit of (u, u_x, u_y) of layer j at (x0, y_line) from above (side = +1) or
        below (-1): values at distances delta, 2 delta, ..., npts delta, extrapolated to
        zero distance by the Lagrange polynomial through them."""
        x0 = np.atleast_1d(np.asarray(x0, float))
        t = delta * np.arange(1, npts + 1)
        tx = np.repeat(x0, npts)
        ty = y_line + side * np.tile(t, len(x0))
        vals = self.layer(j, tx, ty)
        # Lagrange weights of the interpolant through (t_i, v_i) evaluated at 0
        w = np.array([np.prod([t[m] / (t[m] - t[i]) for m in range(npts) if m != i])
                      for i in range(npts)])
        return tuple((v.reshape(len(x0), npts) @ w) for v in vals)
