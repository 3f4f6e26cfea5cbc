"""The empty-structure system A alpha = f (oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 3: the scattered field in each layer is a sum over the near copies
l = -1, 0, 1 of single- and double-layer potentials on the interfaces (phased by
alpha^l) plus a J (Fourier-Bessel) expansion about a centre of the layer
(eqs. repre1-repre3); the unknowns are fixed by continuity of value and normal
derivative across Gamma_1 and Gamma_2 (eq. bound1), quasi-periodicity on the
walls of every layer (eq. bound2) and matching to Rayleigh-Bloch expansions on
Gamma_u, Gamma_d (eq. bound3).  Stacking these rows gives the rectangular
matrix A of eq. matA with right-hand side f of eq. Arhs.

Readings taken here, where the paper is silent or ambiguous:
  * flat interfaces Gamma_1: y = h, Gamma_2: y = -h, normals +y; jump relations
    (S sigma)_n^{+-} = (-+1/2 + N) sigma, (D mu)^{+-} = (+-1/2 + D) mu, "+" above;
  * value rows of an interface are [I + D_diff, S_diff] on (mu, sigma) and normal
    rows [T_diff, -I + N_diff] (differences taken upper minus lower layer); on a
    flat line D = N = 0 identically;
  * the top J expansion enters the Gamma_1 rows and the bottom one the Gamma_2 rows
    (the printed block matrix omits them; the field they represent touches the
    interface, so they are kept);
  * the Gamma_d radiation row uses the bottom-layer field u_3;
  * wall rows use the cancelled form for every three-copy source:
    alpha u(L) - u(L + d) = alpha^2 Phi(L - d) - alpha^{-1} Phi(L + 2d), Phi the l = 0 copy,
    and the x-derivative on both walls;
  * columns of A are equilibrated to unit 2-norm before the pseudo-inverse.

TE polarisation (u = H_z; the paper treats TM only): u and (1/eps) du/dn are
continuous (eps = n^2).  Each layer's potentials carry the factor pv = eps of that
layer and every interface flux row takes (1/eps) d/dn of the field on its side, so
the hypersingular parts still cancel (flux rows keep [T_diff, -I + N_diff]); the
value rows become [(pv_a + pv_b)/2 I + pv_a D_a - pv_b D_b, pv_a S_a - pv_b S_b],
whose single-layer part is now log-singular on the line (weighted difference); J
expansions in flux rows carry 1/eps of their layer.  TM is pv = 1, 1/eps -> 1.

Column order: mu1, sig1, mu2, sig2, a2, a1, a3, c, d.
Row order: Gamma_1 (value, normal), Gamma_2 (value, normal), wall 2 (value,
x-derivative), wall 1, wall 3, Gamma_u (value, y-derivative), Gamma_d.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .common import incoming, grad_wave
from .quadrature import correction_weights


def layer_kernels(k, tx, ty, sx, sy, tdir=None):
    """Free-space single-layer G and double-layer dG/dn_y (n_y = +y) kernels.

    G = (i/4) H_0(k r), dG/dn_y = (i k / 4) H_1(k r) (R . n_y) / r with R = x - y.
    With tdir = (tx_, ty_), return their derivatives along tdir at the target:
      grad_x G . t = -(i k / 4) H_1 (R . t) / r
      grad_x dG/dn_y . t = (i k / 4) [ -k H_2 (R . n_y)(R . t) / r^2 + H_1 (n_y . t) / r ].
    """
    Rx = tx - sx
    Ry = ty - sy
    r = np.hypot(Rx, Ry)
    kr = k * r
    H1 = sp.hankel1(1, kr)
    if tdir is None:
        H0 = sp.hankel1(0, kr)
        return 0.25j * H0, 0.25j * k * H1 * Ry / r
    dx, dy = tdir
    Rt = Rx * dx + Ry * dy
    H2 = sp.hankel1(2, kr)
    dS = -0.25j * k * H1 * Rt / r
    dD = 0.25j * k * (-k * H2 * Ry * Rt / r ** 2 + H1 * dy / r)
    return dS, dD


def _three_copy(G, k, tx, ty, sy_line, tdir=None):
    """Sum over copies l = -1, 0, 1 of the kernels from a line at y = sy_line.

    Targets (tx, ty) are 1-D arrays; returns (S, D) matrices [n_t, N] including
    the trapezoid weight d/N and the phases alpha^l.
    """
    S = 0
    D = 0
    for l in (-1, 0, 1):
        sx = G.xg[None, :] + l * G.d
        a, b = layer_kernels(k, tx[:, None], ty[:, None], sx, np.full_like(sx, sy_line), tdir)
        S = S + G.alpha ** l * a
        D = D + G.alpha ** l * b
    return S * G.hs, D * G.hs


def _wall_cancelled(G, k, yw, sy_line, deriv):
    """Wall discrepancy alpha u(L) - u(R) of a three-copy line source, cancelled form."""
    tdir = (1.0, 0.0) if deriv else None
    out = []
    for xt, wt in ((-1.5 * G.d, G.alpha ** 2), (1.5 * G.d, -G.alpha ** -1)):
        tx = np.full_like(yw, xt)
        a, b = layer_kernels(k, tx[:, None], yw[:, None], G.xg[None, :],
                             np.full((1, G.N), sy_line), tdir)
        out.append((wt * a, wt * b))
    S = (out[0][0] + out[1][0]) * G.hs
    D = (out[0][1] + out[1][1]) * G.hs
    return S, D


def self_kernel_split(ka, kb, wa=1.0, wb=1.0):
    """Log split K(s) = phi(s) ln|s| + psi(s) of the flat-line kernel differences.

    wa S_{ka} - wb S_{kb}: K(s) = (i/4)[wa H_0(ka|s|) - wb H_0(kb|s|)],
        phi(s) = -[wa J_0(ka s) - wb J_0(kb s)] / (2 pi),
        psi(0) = (wa - wb)(i/4 - gamma/(2 pi)) - [wa ln(ka/2) - wb ln(kb/2)] / (2 pi)
        (= -ln(ka/kb) / (2 pi) for wa = wb = 1).
    T_{ka} - T_{kb}: K(s) = (i/4)[ka H_1(ka|s|) - kb H_1(kb|s|)] / |s|,
        phi(s) = -[ka J_1(ka s) - kb J_1(kb s)] / (2 pi s),  phi(0) = -(ka^2 - kb^2) / (4 pi),
        psi(0) = i (ka^2 - kb^2)/8 - [ka^2 ln(ka/2) - kb^2 ln(kb/2)] / (4 pi)
                 + (ka^2 - kb^2)(1 - 2 gamma) / (8 pi),
    from the small-argument series of J_0, Y_0, J_1, Y_1 (the 1/s^2 parts cancel).
    Returns (phiS(s), phiT(s), phiS(0), phiT(0), psiS(0), psiT(0)); phi at s = 0
    returns the limit.
    """
    def phiS(s):
        s = np.abs(np.asarray(s, float))
        return -(wa * sp.j0(ka * s) - wb * sp.j0(kb * s)) / (2 * np.pi)

    def phiT(s):
        s = np.abs(np.asarray(s, float))
        z = s == 0
        ss = np.where(z, 1.0, s)
        v = -(ka * sp.j1(ka * ss) - kb * sp.j1(kb * ss)) / (2 * np.pi * ss)
        return np.where(z, -(ka ** 2 - kb ** 2) / (4 * np.pi), v)

    g = np.euler_gamma
    psiS0 = ((wa - wb) * (0.25j - g / (2 * np.pi))
             - (wa * np.log(ka / 2) - wb * np.log(kb / 2)) / (2 * np.pi))
    psiT0 = (0.125j * (ka ** 2 - kb ** 2)
             - (ka ** 2 * np.log(ka / 2) - kb ** 2 * np.log(kb / 2)) / (4 * np.pi)
             + (ka ** 2 - kb ** 2) * (1 - 2 * g) / (8 * np.pi))
    return (phiS, phiT, -(wa - wb) / (2 * np.pi), -(ka ** 2 - kb ** 2) / (4 * np.pi), psiS0,
            psiT0)


def self_line_blocks(G, ka, kb, wa=1.0, wb=1.0):
    """Same-line blocks wa S_{ka} - wb S_{kb} and T_{ka} - T_{kb} with zeta correction.

    Returns (Sd, Td), each [N, N], acting on the density at the N nodes of the
    central copy; the three copies are folded in with alpha^l.
    """
    N, hs, K = G.N, G.hs, G.pb.disc.zeta_K
    i = np.arange(N)
    Sd = np.zeros((N, N), complex)
    Td = np.zeros((N, N), complex)
    for l in (-1, 0, 1):
        s = G.xg[:, None] - (G.xg[None, :] + l * G.d)
        a = np.abs(s)
        mask = a > 0
        aa = np.where(mask, a, 1.0)
        ks = 0.25j * (wa * sp.hankel1(0, ka * aa) - wb * sp.hankel1(0, kb * aa))
        kt = 0.25j * (ka * sp.hankel1(1, ka * aa) - kb * sp.hankel1(1, kb * aa)) / aa
        ks = np.where(mask, ks, 0)
        kt = np.where(mask, kt, 0)
        Sd += G.alpha ** l * ks * hs
        Td += G.alpha ** l * kt * hs
    # local corrections on the (2K+1)-point stencil around each target
    p = np.arange(-K, K + 1)
    phiS, phiT, phiS0, phiT0, psiS0, psiT0 = self_kernel_split(ka, kb, wa, wb)
    sv = p * hs
    wS = correction_weights(phiS(sv), phiS0, psiS0, hs, K)
    wT = correction_weights(phiT(sv), phiT0, psiT0, hs, K)
    for pi_, pp in enumerate(p):
        gidx = i + pp
        l = np.floor_divide(gidx, N)
        j = gidx - l * N
        ph = G.alpha ** l
        np.add.at(Sd, (i, j), ph * wS[pi_])
        np.add.at(Td, (i, j), ph * wT[pi_])
    return Sd, Td


def _jblock(G, layer, tx, ty, tdir=None):
    """J-expansion columns of a layer (orders -Q..Q) at targets; value or derivative."""
    Q = G.Q[layer]
    k = G.kl[layer]
    cx, cy = G.jc[layer]
    q = np.arange(-Q, Q + 1)[None, :]
    vx = (tx - cx)[:, None]
    vy = (ty - cy)[:, None]
    if tdir is None:
        return incoming(q, k, vx, vy)
    gx, gy = grad_wave(incoming, q, k, vx, vy)
    return gx * tdir[0] + gy * tdir[1]


def assemble_A(G):
    """The rectangular empty-structure matrix A of eq. matA (unscaled columns)."""
    N = G.N
    A = np.zeros((G.n_rows, G.n_alpha), complex)
    R, C = G.row, G.col
    h = G.h
    up = (0.0, 1.0)
    xg = G.xg
    yt1 = np.full(N, h)
    yt2 = np.full(N, -h)
    eye = np.eye(N)
    pv, fl = G.pv, G.fl
    # --- Gamma_1 rows: (u_1 - u_2) and the flux difference (d/dy, times 1/eps for TE)
    Sd1, Td1 = self_line_blocks(G, G.k1, G.k2, pv[0], pv[1])
    A[R["g1v"], C["mu1"]] = 0.5 * (pv[0] + pv[1]) * eye
    A[R["g1v"], C["sig1"]] = Sd1
    A[R["g1n"], C["mu1"]] = Td1
    A[R["g1n"], C["sig1"]] = -eye
    S, D = _three_copy(G, G.k2, xg, yt1, -h)
    A[R["g1v"], C["mu2"]] = -pv[1] * D
    A[R["g1v"], C["sig2"]] = -pv[1] * S
    S, D = _three_copy(G, G.k2, xg, yt1, -h, up)
    A[R["g1n"], C["mu2"]] = -fl[1] * pv[1] * D
    A[R["g1n"], C["sig2"]] = -fl[1] * pv[1] * S
    A[R["g1v"], C["a2"]] = -_jblock(G, 1, xg, yt1)
    A[R["g1n"], C["a2"]] = -fl[1] * _jblock(G, 1, xg, yt1, up)
    A[R["g1v"], C["a1"]] = _jblock(G, 0, xg, yt1)
    A[R["g1n"], C["a1"]] = fl[0] * _jblock(G, 0, xg, yt1, up)
    # --- Gamma_2 rows: (u_2 - u_3) and the flux difference
    Sd2, Td2 = self_line_blocks(G, G.k2, G.k3, pv[1], pv[2])
    S, D = _three_copy(G, G.k2, xg, yt2, h)
    A[R["g2v"], C["mu1"]] = pv[1] * D
    A[R["g2v"], C["sig1"]] = pv[1] * S
    S, D = _three_copy(G, G.k2, xg, yt2, h, up)
    A[R["g2n"], C["mu1"]] = fl[1] * pv[1] * D
    A[R["g2n"], C["sig1"]] = fl[1] * pv[1] * S
    A[R["g2v"], C["mu2"]] = 0.5 * (pv[1] + pv[2]) * eye
    A[R["g2v"], C["sig2"]] = Sd2
    A[R["g2n"], C["mu2"]] = Td2
    A[R["g2n"], C["sig2"]] = -eye
    A[R["g2v"], C["a2"]] = _jblock(G, 1, xg, yt2)
    A[R["g2n"], C["a2"]] = fl[1] * _jblock(G, 1, xg, yt2, up)
    A[R["g2v"], C["a3"]] = -_jblock(G, 2, xg, yt2)
    A[R["g2n"], C["a3"]] = -fl[2] * _jblock(G, 2, xg, yt2, up)
    # --- wall rows: alpha u(L) - u(R), value and x-derivative
    right = (1.0, 0.0)
    for lay, rv, rd, lines in ((1, "w2v", "w2d", ((h, "mu1", "sig1"), (-h, "mu2", "sig2"))),
                               (0, "w1v", "w1d", ((h, "mu1", "sig1"),)),
                               (2, "w3v", "w3d", ((-h, "mu2", "sig2"),))):
        yw = G.yw[lay]
        k = G.kl[lay]
        for deriv, rr in ((False, rv), (True, rd)):
            for ys, cm, cs in lines:
                S, D = _wall_cancelled(G, k, yw, ys, deriv)
                A[R[rr], C[cm]] = pv[lay] * D
                A[R[rr], C[cs]] = pv[lay] * S
            td = right if deriv else None
            JL = _jblock(G, lay, np.full_like(yw, -G.d / 2), yw, td)
            JR = _jblock(G, lay, np.full_like(yw, G.d / 2), yw, td)
            A[R[rr], C[("a1", "a2", "a3")[lay]]] = G.alpha * JL - JR
    # --- Gamma_u rows: u_1 - sum c_n e^{i kappa_n x}, d/dy likewise
    xu = G.xu
    yu = np.full_like(xu, G.y0)
    E = np.exp(1j * G.kapn[None, :] * xu[:, None])
    S, D = _three_copy(G, G.k1, xu, yu, h)
    A[R["uv"], C["mu1"]] = pv[0] * D
    A[R["uv"], C["sig1"]] = pv[0] * S
    S, D = _three_copy(G, G.k1, xu, yu, h, up)
    A[R["un"], C["mu1"]] = pv[0] * D
    A[R["un"], C["sig1"]] = pv[0] * S
    A[R["uv"], C["a1"]] = _jblock(G, 0, xu, yu)
    A[R["un"], C["a1"]] = _jblock(G, 0, xu, yu, up)
    A[R["uv"], C["c"]] = -E
    A[R["un"], C["c"]] = -1j * G.k1n[None, :] * E
    # --- Gamma_d rows: u_3 - sum d_n e^{i kappa_n x}, d/dy likewise
    yd = -yu
    S, D = _three_copy(G, G.k3, xu, yd, -h)
    A[R["dv"], C["mu2"]] = pv[2] * D
    A[R["dv"], C["sig2"]] = pv[2] * S
    S, D = _three_copy(G, G.k3, xu, yd, -h, up)
    A[R["dn"], C["mu2"]] = pv[2] * D
    A[R["dn"], C["sig2"]] = pv[2] * S
    A[R["dv"], C["a3"]] = _jblock(G, 2, xu, yd)
    A[R["dn"], C["a3"]] = _jblock(G, 2, xu, yd, up)
    A[R["dv"], C["d"]] = -E
    A[R["dn"], C["d"]] = 1j * G.k3n[None, :] * E
    return A


def rhs_f(G):
    """Right-hand side f of eq. Arhs: -u_inc and -du_inc/dy (times 1/eps_1 for TE) on
    Gamma_1, zero elsewhere."""
    f = np.zeros(G.n_rows, complex)
    ui = G.u_inc(G.xg, G.h)
    f[G.row["g1v"]] = -ui
    f[G.row["g1n"]] = -G.fl[0] * (-1j * G.k1 * G.cosphi) * ui
    return f
