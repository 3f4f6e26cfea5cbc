"""Scattering matrix of one non-circular inclusion by a boundary integral equation
(oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 4.1 (eqs. rep1, rep2, intg1, intg2 and the formula for s_ln), shapes of
eq. par1.  The inclusion Omega_p (wavenumber k_p inside, k_2 outside) has a smooth
boundary parametrised counter-clockwise by t in [0, 2 pi),

    gamma(t) = rho(t) (cos(t + rot), sin(t + rot)),  rho(t) = a1 + a2 cos(a3 t),

so its outward normal is n = (gamma_y', -gamma_x') / |gamma'|.  With
G_k(x, y) = (i/4) H_0(k |x - y|) and the layer potentials

    S_k sigma = int G_k sigma ds_y,            D_k mu = int dG_k/dn_y mu ds_y,
    N_k sigma = int dG_k/dn_x sigma ds_y,      T_k mu = int d^2 G_k/dn_x dn_y mu ds_y,

the exterior scattered field is u^s = S_{k2} sigma + D_{k2} mu and the interior
field u = S_{kp} sigma + D_{kp} mu (eqs. rep1, rep2).  Continuity of u and du/dn
across the boundary with the jump relations (exterior limit of D: D mu + mu/2,
interior D mu - mu/2; of dS/dn: N sigma -/+ sigma/2) gives the second-kind system
of eqs. intg1 and intg2,

     mu + (S_{k2} - S_{kp}) sigma + (D_{k2} - D_{kp}) mu = -u_inc,
    -sigma + (N_{k2} - N_{kp}) sigma + (T_{k2} - T_{kp}) mu = -du_inc/dn.

For the incoming wave u_inc = J_n(k2 r) e^{i n theta} (about the centre) the
outgoing coefficients follow from Graf's theorem for |x| > |y|,
H_0(k|x - y|) = sum_l H_l(k|x|) e^{il theta_x} J_l(k|y|) e^{-il theta_y}:

    s_ln = (i/4) int [ J_l(k2|y|) e^{-il theta_y} sigma_n(y)
                       + dn_y (J_l(k2|y|) e^{-il theta_y}) mu_n(y) ] ds_y.

(Reading: the paper prints this formula without the factor i/4; here the layer
potentials carry the free-space Green's function (i/4) H_0, and the factor is the
one Graf's theorem gives for it.)

Quadrature: Kress' product rule for 2 pi-periodic kernels with a logarithmic
singularity (R. Kress, Boundary integral equations in time-harmonic acoustic
scattering, Math. Comput. Modelling 15 (1991); Colton and Kress, Inverse Acoustic
and Electromagnetic Scattering Theory, sec. 3.5).  Each kernel difference is split
as K(t, tau) = K1(t, tau) ln(4 sin^2((t - tau)/2)) + K2(t, tau) with smooth K1, K2;
on 2n nodes t_j = j pi / n,

    int_0^{2pi} K(t_i, tau) phi(tau) dtau
        ~ sum_j [ R_{i-j} K1(t_i, t_j) + (pi / n) K2(t_i, t_j) ] phi(t_j),
    R_m = -(2 pi / n) sum_{q=1}^{n-1} cos(q m pi / n) / q - (pi / n^2) cos(m pi).

K1 is the coefficient of ln |x - y|^2: replacing (i/4) H_m(kr) by -(1/(4 pi)) J_m(kr) in each kernel.  The
diagonal values K2(t, t) of the differences come from the small-r expansions
(i/4) H_0(kr) = -(1/(2 pi)) J_0(kr) ln r + R_0(kr), R_0 an even power series,
with c(k) = ln(k/2) + Euler's gamma:

    S_{k1} - S_{k2}:  K1(t, t) = 0,   K2(t, t) = -ln(k1/k2) / (2 pi),
    D and N differences: both 0,
    T_{k1} - T_{k2}:  K1(t, t) = -a,  K2(t, t) = -a - 2 b - a ln|gamma'(t)|^2,
        a = (k1^2 - k2^2) / (8 pi),
        b = -(i/16)(k1^2 - k2^2) + (k1^2 c(k1) - k2^2 c(k2)) / (8 pi) - (k1^2 - k2^2) / (8 pi),

all times the speed |gamma'(tau)| of the parametrisation.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

EULER = 0.5772156649015329


def curve(a1, a2, a3, rot, t):
    """Points, first derivatives and speed of the boundary at parameters t."""
    rho = a1 + a2 * np.cos(a3 * t)
    drho = -a2 * a3 * np.sin(a3 * t)
    c, s = np.cos(t + rot), np.sin(t + rot)
    x, y = rho * c, rho * s
    dx, dy = drho * c - rho * s, drho * s + rho * c
    return x, y, dx, dy, np.hypot(dx, dy)


def kress_weights(n):
    """R_m, m = 0 .. 2n-1, of Kress' rule on 2n nodes (the weight of node j for the
    target i is R_{(i - j) mod 2n})."""
    m = np.arange(2 * n)
    t = m * np.pi / n
    q = np.arange(1, n)
    return (-(2 * np.pi / n) * (np.cos(np.outer(t, q)) / q[None, :]).sum(axis=1)
            - (np.pi / n ** 2) * np.cos(n * t))


def _h(m, z):
    return sp.hankel1(m, z)


def kernel_blocks(k, X, Y, NX, NY):
    """The four kernels at target points X (with normals NX) and source points Y
    (normals NY), off the diagonal: (S, D, N, T) values and their ln|x-y|^2
    coefficients (S1, D1, N1, T1).  Arrays [targets, sources]."""
    Rx = X[:, None, 0] - Y[None, :, 0]
    Ry = X[:, None, 1] - Y[None, :, 1]
    r = np.hypot(Rx, Ry)
    z = k * r
    rnx = Rx * NX[:, None, 0] + Ry * NX[:, None, 1]      # R . n_x
    rny = Rx * NY[None, :, 0] + Ry * NY[None, :, 1]      # R . n_y
    nxny = NX[:, None, 0] * NY[None, :, 0] + NX[:, None, 1] * NY[None, :, 1]
    H0, H1, H2 = _h(0, z), _h(1, z), _h(2, z)
    J0, J1, J2 = sp.jv(0, z), sp.jv(1, z), sp.jv(2, z)
    S = 0.25j * H0
    D = 0.25j * k * H1 * rny / r
    N = -0.25j * k * H1 * rnx / r
    T = 0.25j * k * (-k * H2 * rnx * rny / r ** 2 + H1 * nxny / r)
    c = -1.0 / (4 * np.pi)
    S1 = c * J0
    D1 = c * k * J1 * rny / r
    N1 = -c * k * J1 * rnx / r
    T1 = c * k * (-k * J2 * rnx * rny / r ** 2 + J1 * nxny / r)
    return (S, D, N, T), (S1, D1, N1, T1)


def bie_system(a1, a2, a3, rot, k2, kp, n):
    """The matrix of eqs. intg1, intg2 on 2n nodes, unknowns [mu; sigma] at the
    nodes, rows [intg1; intg2]; also the nodes, normals and quadrature speeds."""
    N2 = 2 * n
    t = np.arange(N2) * np.pi / n
    x, y, dx, dy, sp_ = curve(a1, a2, a3, rot, t)
    P = np.stack([x, y], axis=1)
    Nrm = np.stack([dy, -dx], axis=1) / sp_[:, None]
    R = kress_weights(n)
    idx = (np.arange(N2)[:, None] - np.arange(N2)[None, :]) % N2
    Rm = R[idx]
    off = ~np.eye(N2, dtype=bool)
    L = np.zeros((N2, N2))
    tt = t[:, None] - t[None, :]
    L[off] = np.log(4 * np.sin(tt[off] / 2) ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        (Sa, Da, Na, Ta), (S1a, D1a, N1a, T1a) = kernel_blocks(k2, P, P, Nrm, Nrm)
        (Sb, Db, Nb, Tb), (S1b, D1b, N1b, T1b) = kernel_blocks(kp, P, P, Nrm, Nrm)
    blocks = {}
    for name, Ka, Kb, K1a, K1b in (("S", Sa, Sb, S1a, S1b), ("D", Da, Db, D1a, D1b),
                                    ("N", Na, Nb, N1a, N1b), ("T", Ta, Tb, T1a, T1b)):
        K = np.where(off, Ka - Kb, 0.0)
        K1 = np.where(off, K1a - K1b, 0.0)
        K2 = np.where(off, K - K1 * L, 0.0)
        blocks[name] = [K1, K2]
    # diagonal limits of the differences (module docstring)
    d = np.arange(N2)
    blocks["S"][1][d, d] = -np.log(k2 / kp) / (2 * np.pi)
    ca = (k2 ** 2 - kp ** 2) / (8 * np.pi)
    cb = (-(1j / 16) * (k2 ** 2 - kp ** 2)
          + (k2 ** 2 * (np.log(k2 / 2) + EULER) - kp ** 2 * (np.log(kp / 2) + EULER)) / (8 * np.pi)
          - (k2 ** 2 - kp ** 2) / (8 * np.pi))
    blocks["T"][0][d, d] = -ca
    blocks["T"][1][d, d] = -ca - 2 * cb - ca * np.log(sp_ ** 2)
    W = {}
    for name, (K1, K2) in blocks.items():
        W[name] = (Rm * K1 + (np.pi / n) * K2) * sp_[None, :]
    I = np.eye(N2)
    A = np.block([[I + W["D"], W["S"]], [W["T"], -I + W["N"]]])
    return A, P, Nrm, sp_


def _jwave(m, k, X):
    """J_m(k|x|) e^{i m theta_x} at points X [.., 2]."""
    r = np.hypot(X[..., 0], X[..., 1])
    th = np.arctan2(X[..., 1], X[..., 0])
    return sp.jv(m, k * r) * np.exp(1j * m * th)


def _jwave_grad(m, k, X):
    """(d/dx, d/dy) of J_m(k|x|) e^{i m theta} by (d_x +- i d_y) Z_m e^{im theta}
    = -+ k Z_{m+-1} e^{i(m+-1) theta}."""
    fm, fp = _jwave(m - 1, k, X), _jwave(m + 1, k, X)
    return 0.5 * k * (fm - fp), 0.5j * k * (fm + fp)


def scattering_matrix(a1, a2, a3, rot, k2, kp, P, n=64):
    """s_ln, l, n = -P..P (index + P), of the inclusion of eq. par1 rotated by rot,
    from the BIE on 2n boundary nodes."""
    A, X, Nrm, spd = bie_system(a1, a2, a3, rot, k2, kp, n)
    N2 = 2 * n
    orders = np.arange(-P, P + 1)
    rhs = np.zeros((2 * N2, orders.size), complex)
    for c, m in enumerate(orders):
        gx, gy = _jwave_grad(m, k2, X)
        rhs[:N2, c] = -_jwave(m, k2, X)
        rhs[N2:, c] = -(gx * Nrm[:, 0] + gy * Nrm[:, 1])
    sol = np.linalg.solve(A, rhs)
    mu, sig = sol[:N2], sol[N2:]
    w = (np.pi / n) * spd                      # trapezoid weights times speed
    S = np.zeros((orders.size, orders.size), complex)
    for r_, l in enumerate(orders):
        # W_l(y) = J_l(k2|y|) e^{-il theta_y} = (-1)^l J_{-l}(k2|y|) e^{i(-l) theta_y}
        sgn = (-1.0) ** l
        Wl = sgn * _jwave(-l, k2, X)
        gx, gy = _jwave_grad(-l, k2, X)
        dWl = sgn * (gx * Nrm[:, 0] + gy * Nrm[:, 1])
        S[r_, :] = 0.25j * ((w * Wl) @ sig + (w * dWl) @ mu)
    return S


def scattered_field_direct(a1, a2, a3, rot, k2, kp, n, m, X):
    """u^s = S_{k2} sigma + D_{k2} mu at exterior points X [npts, 2] for the
    incoming wave J_m(k2 r) e^{im theta}, by the trapezoid rule on the densities
    (accurate for points well away from the boundary)."""
    A, Y, Nrm, spd = bie_system(a1, a2, a3, rot, k2, kp, n)
    N2 = 2 * n
    gx, gy = _jwave_grad(m, k2, Y)
    rhs = np.concatenate([-_jwave(m, k2, Y), -(gx * Nrm[:, 0] + gy * Nrm[:, 1])])
    sol = np.linalg.solve(A, rhs)
    mu, sig = sol[:N2], sol[N2:]
    (S, D, _, _), _ = kernel_blocks(k2, np.asarray(X, float), Y, np.zeros_like(X), Nrm)
    w = (np.pi / n) * spd
    return S @ (w * sig) + D @ (w * mu)


def rotate_matrix(S, rot):
    """Scattering matrix of the same inclusion turned counter-clockwise by rot:
    incoming coefficients seen by the turned inclusion are a_n e^{in rot}, its
    outgoing ones b_l e^{-il rot}, so S'_ln = e^{i rot (n - l)} s_ln (the paper's
    phase factor with the opposite sense of rotation)."""
    P = (S.shape[0] - 1) // 2
    o = np.arange(-P, P + 1)
    return np.exp(1j * rot * (o[None, :] - o[:, None])) * S
