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
  * interfaces are graphs y = f_j(x) of period d (flat: f = +-h), parametrised by
    x with equispaced nodes, normals pointing up; jump relations
    (S sigma)_n^{+-} = (-+1/2 + N) sigma, (D mu)^{+-} = (+-1/2 + D) mu, "+" above;
  * value rows of an interface are [I + D_diff, S_diff] on (mu, sigma) and normal
    rows [T_diff, -I + N_diff] (differences taken upper minus lower layer); on a
    flat line D = N = 0 identically;
  * the same-interface blocks use the zeta-corrected trapezoid rule (in place of
    the paper's Alpert corrections, whose tables are not printed) per target, on
    the kernels' log split in the parameter x, the stencil wrapping onto the
    neighbouring copies with their Bloch phases;
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


def layer_kernels(k, tx, ty, sx, sy, tdir=None, snrm=(0.0, 1.0)):
    """Free-space single-layer G and double-layer dG/dn_y kernels (source normal
    snrm), R = x - y:
      G = (i/4) H_0(k r),  dG/dn_y = (i k / 4) H_1(k r) (R . n_y) / r.
    With tdir = (tx_, ty_), return their derivatives along tdir at the target:
      grad_x G . t = -(i k / 4) H_1 (R . t) / r
      grad_x dG/dn_y . t = (i k / 4) [ -k H_2 (R . n_y)(R . t) / r^2 + H_1 (n_y . t) / r ].
    """
    Rx = tx - sx
    Ry = ty - sy
    r = np.hypot(Rx, Ry)
    kr = k * r
    H1 = sp.hankel1(1, kr)
    Rn = Rx * snrm[0] + Ry * snrm[1]
    if tdir is None:
        H0 = sp.hankel1(0, kr)
        return 0.25j * H0, 0.25j * k * H1 * Rn / r
    dx, dy = tdir
    Rt = Rx * dx + Ry * dy
    H2 = sp.hankel1(2, kr)
    dS = -0.25j * k * H1 * Rt / r
    dD = 0.25j * k * (-k * H2 * Rn * Rt / r ** 2 + H1 * (snrm[0] * dx + snrm[1] * dy) / r)
    return dS, dD


def _tcol(tdir, n):
    """A target direction (scalars or per-target arrays) as [n, 1] columns."""
    if tdir is None:
        return None
    return tuple(np.broadcast_to(np.asarray(t, float), (n,))[:, None] for t in tdir)


def _line_sources(G, line):
    """Source nodes of interface `line` (0: Gamma_1, 1: Gamma_2) as [1, N] rows:
    x, y, normal, arc-length weight."""
    return (G.xg[None, :], G.gy[line][None, :],
            (G.gn[line][0][None, :], G.gn[line][1][None, :]), G.gw[line][None, :])


def _three_copy(G, k, tx, ty, line, tdir=None):
    """Sum over copies l = -1, 0, 1 of the kernels from interface `line`.

    Targets (tx, ty) are 1-D arrays (tdir: scalars or per-target arrays); returns
    (S, D) matrices [n_t, N] including the arc-length weights and the phases alpha^l.
    """
    sx, sy, sn, sw = _line_sources(G, line)
    td = _tcol(tdir, len(tx))
    S = 0
    D = 0
    for l in (-1, 0, 1):
        a, b = layer_kernels(k, tx[:, None], ty[:, None], sx + l * G.d, sy, td, sn)
        S = S + G.alpha ** l * a
        D = D + G.alpha ** l * b
    return S * sw, D * sw


def _wall_cancelled(G, k, yw, line, deriv):
    """Wall discrepancy alpha u(L) - u(R) of a three-copy interface source,
    cancelled form."""
    tdir = (1.0, 0.0) if deriv else None
    sx, sy, sn, sw = _line_sources(G, line)
    out = []
    for xt, wt in ((-1.5 * G.d, G.alpha ** 2), (1.5 * G.d, -G.alpha ** -1)):
        tx = np.full_like(yw, xt)
        a, b = layer_kernels(k, tx[:, None], yw[:, None], sx, sy, tdir, sn)
        out.append((wt * a, wt * b))
    S = (out[0][0] + out[1][0]) * sw
    D = (out[0][1] + out[1][1]) * sw
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
    returns the limit.  This is the flat case (speed 1, no curvature) of
    curve_kernel_limits.
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

    lim = curve_kernel_limits(ka, kb, wa, wb, 1.0, 0.0)
    return phiS, phiT, lim["S"][0], lim["T"][0], lim["S"][1], lim["T"][1]


def curve_kernel_limits(ka, kb, wa, wb, spd, f2):
    """(phi(0), psi(0)) of the four same-interface kernel differences on a graph
    y = f(x) in the parameter x, at a node with speed spd = |(1, f')| and f'' = f2.

    Each kernel per unit of the source parameter t splits as
    K(s, t) = phi(s, t) ln|s - t| + psi(s, t) (ln r = ln|s - t| + ln spd + O(s - t));
    the log coefficient of (i/4) H_n(k r) is -J_n(k r) / (2 pi), and the k-free
    singular parts (1/(2 pi r) of (i/4) k H_1, 1/r^2 of the T kernel) cancel in the
    differences except for the weighted double layer, whose part
    (R . n_t) / (2 pi r^2) tends to f'' / (4 pi spd^3) per unit length.
      S: wa S_a - wb S_b   phi0 = -(wa - wb) spd / (2 pi)
         psi0 = spd [(wa - wb)(i/4 - gamma/(2 pi) - ln(spd)/(2 pi)) - (wa ln(ka/2) - wb ln(kb/2))/(2 pi)]
      D: wa D_a - wb D_b   phi0 = 0, psi0 = (wa - wb) f'' / (4 pi spd^2)
      N: N_a - N_b         phi0 = 0, psi0 = 0
      T: T_a - T_b         phi0 = -(ka^2 - kb^2) spd / (4 pi)
         psi0 = spd [i (ka^2 - kb^2)/8 - (ka^2 ln(ka/2) - kb^2 ln(kb/2))/(4 pi)
                     + (ka^2 - kb^2)(1 - 2 gamma)/(8 pi) - (ka^2 - kb^2) ln(spd)/(4 pi)]
    """
    g = np.euler_gamma
    d2 = ka ** 2 - kb ** 2
    lsp = np.log(spd)
    S = (-(wa - wb) * spd / (2 * np.pi),
         spd * ((wa - wb) * (0.25j - g / (2 * np.pi) - lsp / (2 * np.pi))
                - (wa * np.log(ka / 2) - wb * np.log(kb / 2)) / (2 * np.pi)))
    D = (0.0, (wa - wb) * f2 / (4 * np.pi * spd ** 2))
    Nn = (0.0, 0.0)
    T = (-d2 * spd / (4 * np.pi),
         spd * (0.125j * d2 - (ka ** 2 * np.log(ka / 2) - kb ** 2 * np.log(kb / 2)) / (4 * np.pi)
                + d2 * (1 - 2 * g) / (8 * np.pi) - d2 * lsp / (4 * np.pi)))
    return {"S": S, "D": D, "N": Nn, "T": T}


def curve_kernels(ka, kb, wa, wb, Rx, Ry, ns, nt, spd_t):
    """The four kernel differences per unit of the source parameter, and their log
    coefficients phi, at R = target - source (r > 0), target normal ns, source
    normal nt, source speed spd_t.  Returns {kind: (K, phi)} for kind in S, D, N, T:
      S = (i/4)(wa H0_a - wb H0_b)
      D = (i/4)(wa ka H1_a - wb kb H1_b)(R . n_t)/r
      N = -(i/4)(ka H1_a - kb H1_b)(R . n_s)/r
      T = (i/4)[(ka H1_a - kb H1_b)(n_s . n_t)/r - (ka^2 H2_a - kb^2 H2_b)(R . n_s)(R . n_t)/r^2]
    each times spd_t; phi is the same expression with (i/4) H_n replaced by its log
    coefficient -J_n / (2 pi)."""
    r = np.hypot(Rx, Ry)
    Rs = Rx * ns[0] + Ry * ns[1]
    Rt = Rx * nt[0] + Ry * nt[1]
    nn = ns[0] * nt[0] + ns[1] * nt[1]
    out = {}
    for kind in ("K", "phi"):
        if kind == "K":
            Z = lambda n, k: 0.25j * sp.hankel1(n, k * r)
        else:
            Z = lambda n, k: -sp.jv(n, k * r) / (2 * np.pi)
        S = (wa * Z(0, ka) - wb * Z(0, kb)) * spd_t
        D = (wa * ka * Z(1, ka) - wb * kb * Z(1, kb)) * Rt / r * spd_t
        Nk = -(ka * Z(1, ka) - kb * Z(1, kb)) * Rs / r * spd_t
        T = ((ka * Z(1, ka) - kb * Z(1, kb)) * nn / r
             - (ka ** 2 * Z(2, ka) - kb ** 2 * Z(2, kb)) * Rs * Rt / r ** 2) * spd_t
        out[kind] = {"S": S, "D": D, "N": Nk, "T": T}
    return {q: (out["K"][q], out["phi"][q]) for q in ("S", "D", "N", "T")}


def self_blocks(G, line, ka, kb, wa=1.0, wb=1.0):
    """Same-interface blocks of interface `line`: wa S_a - wb S_b, wa D_a - wb D_b,
    N_a - N_b and T_a - T_b with zeta-corrected trapezoid weights per target.

    Returns {kind: [N, N]} acting on the density at the N nodes of the central copy;
    the three copies are folded in with alpha^l.  The local correction around each
    target takes phi at the 2K + 1 stencil nodes (which may lie on a neighbouring
    copy, then with its Bloch phase) and phi(0), psi(0) of curve_kernel_limits.
    """
    N, hs, K = G.N, G.hs, G.pb.disc.zeta_K
    x, y = G.xg, G.gy[line]
    ns = G.gn[line]
    spd = G.sp[line]
    out = {q: np.zeros((N, N), complex) for q in ("S", "D", "N", "T")}
    for l in (-1, 0, 1):
        Rx = x[:, None] - (x[None, :] + l * G.d)
        Ry = y[:, None] - y[None, :]
        selfm = (l == 0) & np.eye(N, dtype=bool)
        Rx = np.where(selfm, 1.0, Rx)   # placeholder on the punctured diagonal
        kv = curve_kernels(ka, kb, wa, wb, Rx, Ry, (ns[0][:, None], ns[1][:, None]),
                           (ns[0][None, :], ns[1][None, :]), spd[None, :])
        for q in out:
            out[q] += G.alpha ** l * np.where(selfm, 0.0, kv[q][0]) * hs
    p = np.arange(-K, K + 1)
    for i in range(N):
        gidx = i + p
        lc = np.floor_divide(gidx, N)
        j = gidx - lc * N
        Rx = x[i] - (x[j] + lc * G.d)
        Ry = y[i] - y[j]
        ctr = p == 0
        Rx = np.where(ctr, 1.0, Rx)
        kv = curve_kernels(ka, kb, wa, wb, Rx, Ry, (ns[0][i], ns[1][i]),
                           (ns[0][j], ns[1][j]), spd[j])
        lim = curve_kernel_limits(ka, kb, wa, wb, spd[i], G.gd2[line][i])
        ph = G.alpha ** lc
        for q in out:
            phi = np.where(ctr, lim[q][0], kv[q][1])
            w = correction_weights(phi, lim[q][0], lim[q][1], hs, K)
            np.add.at(out[q], (np.full_like(j, i), j), ph * w)
    return out


def _jblock(G, layer, tx, ty, tdir=None):
    """J-expansion columns of a layer (orders -Q..Q) at targets; value or derivative
    along tdir (scalars or per-target arrays)."""
    Q = G.Q[layer]
    k = G.kl[layer]
    cx, cy = G.jc[layer]
    q = np.arange(-Q, Q + 1)[None, :]
    vx = (tx - cx)[:, None]
    vy = (ty - cy)[:, None]
    if tdir is None:
        return incoming(q, k, vx, vy)
    gx, gy = grad_wave(incoming, q, k, vx, vy)
    td = _tcol(tdir, len(tx))
    return gx * td[0] + gy * td[1]


def assemble_A(G):
    """The rectangular empty-structure matrix A of eq. matA (unscaled columns)."""
    N = G.N
    A = np.zeros((G.n_rows, G.n_alpha), complex)
    R, C = G.row, G.col
    up = (0.0, 1.0)
    xg = G.xg
    yt1, yt2 = G.gy
    n1, n2 = G.gn
    eye = np.eye(N)
    pv, fl = G.pv, G.fl
    # --- Gamma_1 rows: (u_1 - u_2) and the flux difference (d/dn, times 1/eps for TE)
    sb = self_blocks(G, 0, G.k1, G.k2, pv[0], pv[1])
    A[R["g1v"], C["mu1"]] = 0.5 * (pv[0] + pv[1]) * eye + sb["D"]
    A[R["g1v"], C["sig1"]] = sb["S"]
    A[R["g1n"], C["mu1"]] = sb["T"]
    A[R["g1n"], C["sig1"]] = -eye + sb["N"]
    S, D = _three_copy(G, G.k2, xg, yt1, 1)
    A[R["g1v"], C["mu2"]] = -pv[1] * D
    A[R["g1v"], C["sig2"]] = -pv[1] * S
    S, D = _three_copy(G, G.k2, xg, yt1, 1, n1)
    A[R["g1n"], C["mu2"]] = -fl[1] * pv[1] * D
    A[R["g1n"], C["sig2"]] = -fl[1] * pv[1] * S
    A[R["g1v"], C["a2"]] = -_jblock(G, 1, xg, yt1)
    A[R["g1n"], C["a2"]] = -fl[1] * _jblock(G, 1, xg, yt1, n1)
    A[R["g1v"], C["a1"]] = _jblock(G, 0, xg, yt1)
    A[R["g1n"], C["a1"]] = fl[0] * _jblock(G, 0, xg, yt1, n1)
    # --- Gamma_2 rows: (u_2 - u_3) and the flux difference
    sb = self_blocks(G, 1, G.k2, G.k3, pv[1], pv[2])
    S, D = _three_copy(G, G.k2, xg, yt2, 0)
    A[R["g2v"], C["mu1"]] = pv[1] * D
    A[R["g2v"], C["sig1"]] = pv[1] * S
    S, D = _three_copy(G, G.k2, xg, yt2, 0, n2)
    A[R["g2n"], C["mu1"]] = fl[1] * pv[1] * D
    A[R["g2n"], C["sig1"]] = fl[1] * pv[1] * S
    A[R["g2v"], C["mu2"]] = 0.5 * (pv[1] + pv[2]) * eye + sb["D"]
    A[R["g2v"], C["sig2"]] = sb["S"]
    A[R["g2n"], C["mu2"]] = sb["T"]
    A[R["g2n"], C["sig2"]] = -eye + sb["N"]
    A[R["g2v"], C["a2"]] = _jblock(G, 1, xg, yt2)
    A[R["g2n"], C["a2"]] = fl[1] * _jblock(G, 1, xg, yt2, n2)
    A[R["g2v"], C["a3"]] = -_jblock(G, 2, xg, yt2)
    A[R["g2n"], C["a3"]] = -fl[2] * _jblock(G, 2, xg, yt2, n2)
    # --- wall rows: alpha u(L) - u(R), value and x-derivative
    right = (1.0, 0.0)
    for lay, rv, rd, lines in ((1, "w2v", "w2d", ((0, "mu1", "sig1"), (1, "mu2", "sig2"))),
                               (0, "w1v", "w1d", ((0, "mu1", "sig1"),)),
                               (2, "w3v", "w3d", ((1, "mu2", "sig2"),))):
        yw = G.yw[lay]
        k = G.kl[lay]
        for deriv, rr in ((False, rv), (True, rd)):
            for line, cm, cs in lines:
                S, D = _wall_cancelled(G, k, yw, line, deriv)
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
    S, D = _three_copy(G, G.k1, xu, yu, 0)
    A[R["uv"], C["mu1"]] = pv[0] * D
    A[R["uv"], C["sig1"]] = pv[0] * S
    S, D = _three_copy(G, G.k1, xu, yu, 0, up)
    A[R["un"], C["mu1"]] = pv[0] * D
    A[R["un"], C["sig1"]] = pv[0] * S
    A[R["uv"], C["a1"]] = _jblock(G, 0, xu, yu)
    A[R["un"], C["a1"]] = _jblock(G, 0, xu, yu, up)
    A[R["uv"], C["c"]] = -E
    A[R["un"], C["c"]] = -1j * G.k1n[None, :] * E
    # --- Gamma_d rows: u_3 - sum d_n e^{i kappa_n x}, d/dy likewise
    yd = -yu
    S, D = _three_copy(G, G.k3, xu, yd, 1)
    A[R["dv"], C["mu2"]] = pv[2] * D
    A[R["dv"], C["sig2"]] = pv[2] * S
    S, D = _three_copy(G, G.k3, xu, yd, 1, up)
    A[R["dn"], C["mu2"]] = pv[2] * D
    A[R["dn"], C["sig2"]] = pv[2] * S
    A[R["dv"], C["a3"]] = _jblock(G, 2, xu, yd)
    A[R["dn"], C["a3"]] = _jblock(G, 2, xu, yd, up)
    A[R["dv"], C["d"]] = -E
    A[R["dn"], C["d"]] = 1j * G.k3n[None, :] * E
    return A


def rhs_f(G):
    """Right-hand side f of eq. Arhs: -u_inc and -du_inc/dn (times 1/eps_1 for TE) on
    Gamma_1, zero elsewhere."""
    f = np.zeros(G.n_rows, complex)
    ui = G.u_inc(G.xg, G.gy[0])
    nx, ny = G.gn[0]
    f[G.row["g1v"]] = -ui
    f[G.row["g1n"]] = -G.fl[0] * 1j * (G.kappa * nx - G.k1 * G.cosphi * ny) * ui
    return f
