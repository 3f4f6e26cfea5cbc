"""Single-disk scattering matrices and the translation operator (oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 4.1: for a disk the scattering matrix is diagonal; with incoming
J_n(k_2 r) e^{in theta} and outgoing s_n H_n(k_2 r) e^{in theta} outside, and
c_n J_n(k_p r) e^{in theta} inside, continuity of value and radial derivative at
r = R gives (TM, constant mu)

    s_n = -[k_2 J_n'(x) J_n(y) - k_p J_n(x) J_n'(y)] / [k_2 H_n'(x) J_n(y) - k_p H_n(x) J_n'(y)],

x = k_2 R, y = k_p R, and s_{-n} = s_n.

Paper sec. 4.2 / sec. 5: the translation (M2L) operator maps the outgoing
coefficients of inclusion m and of its near copies at x_m + l d (phase alpha^l,
l = -1, 0, 1, eq. repre3_mod) to incoming coefficients about inclusion j.  By
Graf's addition theorem

    H_nu(k|x - c_m|) e^{i nu theta(x - c_m)}
        = sum_n H_{nu-n}(k rho) e^{i (nu-n) phi} J_n(k|x - c_j|) e^{i n theta(x - c_j)},

rho e^{i phi} = c_j - c_m, valid for |x - c_j| < rho, so the block is

    T[(j, n), (m, nu)] = sum_{l, (j,m,l) != (j,j,0)} alpha^l H_{nu-n}(k_2 rho_l) e^{i (nu-n) phi_l},
    rho_l e^{i phi_l} = c_j - c_m - l d e_x.

The far copies |l| >= 2 are not in T: their field is carried by the middle-layer
J expansion.  H_q comes from SciPy (AMOS), not from a recurrence.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def mie_coefficients(k2, kp, R, P, eps2=None, epsp=None):
    """s_n, n = -P..P, for disks (arrays kp, R of length M) -> [M, 2P+1].

    TM: u and du/dr continuous at r = R.  With eps2, epsp given (TE: u and
    (1/eps) du/dr continuous) the radial derivatives are weighted by 1/eps.  kp (and
    epsp) may be complex: absorbing disks."""
    kp = np.atleast_1d(np.asarray(kp))
    R = np.atleast_1d(np.asarray(R, float))
    n = np.arange(0, P + 1)[None, :]
    x = (k2 * R)[:, None]
    y = (kp * R)[:, None]
    w2 = k2 if eps2 is None else k2 / eps2
    kpp = (kp if epsp is None else kp / np.atleast_1d(np.asarray(epsp)))[:, None]
    num = w2 * sp.jvp(n, x) * sp.jv(n, y) - kpp * sp.jv(n, x) * sp.jvp(n, y)
    den = w2 * sp.h1vp(n, x) * sp.jv(n, y) - kpp * sp.hankel1(n, x) * sp.jvp(n, y)
    s = -num / den
    return np.concatenate([s[:, :0:-1], s], axis=1)


def image_displacements(G, j, m):
    """(dx, dy, weight) of the image pairs contributing to T[j, m] (arrays over l)."""
    out = []
    for l in (-1, 0, 1):
        if j == m and l == 0:
            continue
        out.append((G.cx[j] - G.cx[m] - l * G.d, G.cy[j] - G.cy[m], G.alpha ** l))
    return out


def generator(G, jlist):
    """tau[j, m, q] = sum_l alpha^l H_q(k_2 rho_l) e^{i q phi_l}, q = -2P..2P.

    Returns [len(jlist), M, 4P+1]; the excluded self term (j = m, l = 0) is absent.
    """
    P, M = G.P, G.M
    jl = np.asarray(jlist)
    q = np.arange(0, 2 * P + 1)
    tau = np.zeros((len(jl), M, 4 * P + 1), complex)
    sgn = (-1.0) ** q
    for l in (-1, 0, 1):
        dx = G.cx[jl][:, None] - G.cx[None, :] - l * G.d
        dy = G.cy[jl][:, None] - G.cy[None, :] + 0 * dx
        r = np.hypot(dx, dy)
        self_ = r == 0
        rr = np.where(self_, 1.0, r)
        H = sp.hankel1(q[None, None, :], G.k2 * rr[:, :, None])
        e = (dx + 1j * dy) / rr
        th = np.angle(e)
        ep = np.exp(1j * q[None, None, :] * th[:, :, None])
        pos = H * ep                       # q >= 0
        neg = sgn * H * np.conj(ep)        # H_{-q} e^{-i q phi}
        w = np.where(self_, 0.0, 1.0)[:, :, None] * G.alpha ** l
        tau[:, :, 2 * P:] += w * pos
        tau[:, :, :2 * P] += (w * neg)[:, :, :0:-1]  # orders -2P..-1
    return tau


def dense_T(G):
    """Dense T of size [M(2P+1), M(2P+1)] (small M only)."""
    P, M = G.P, G.M
    nb = 2 * P + 1
    tau = generator(G, np.arange(M))
    n = np.arange(-P, P + 1)
    qidx = (n[None, :] - n[:, None]) + 2 * P      # index of nu - n, rows n, cols nu
    T = tau[:, :, qidx]                           # [j, m, n, nu]
    return T.transpose(0, 2, 1, 3).reshape(M * nb, M * nb)


class TranslationTable:
    """Matrix-free application of T from a stored generator table (large M).

    rows: the target inclusions whose rows of T are kept (default all); apply then
    returns alpha^T for those targets only."""

    def __init__(self, G, chunk=64, rows=None):
        self.G = G
        M = G.M
        self.rows = np.arange(M) if rows is None else np.asarray(rows)
        self.tau = np.empty((len(self.rows), M, 4 * G.P + 1), complex)
        for a in range(0, len(self.rows), chunk):
            js = self.rows[a:a + chunk]
            self.tau[a:a + len(js)] = generator(G, js)

    def apply(self, beta):
        """alpha^T[j, n] = sum_m sum_q tau[j, m, q] beta[m, n + q]."""
        G = self.G
        P = G.P
        b = np.asarray(beta).reshape(G.M, 2 * P + 1)
        out = np.zeros((len(self.rows), 2 * P + 1), complex)
        for qi in range(4 * P + 1):
            q = qi - 2 * P
            n_lo = max(-P, -P - q)
            n_hi = min(P, P - q)
            if n_lo > n_hi:
                continue
            out[:, n_lo + P:n_hi + P + 1] += self.tau[:, :, qi] @ b[:, n_lo + q + P:n_hi + q + P + 1]
        return out.reshape(-1)


def apply_T_rows(G, beta, jlist):
    """alpha^T for a few targets only (used to sample large problems)."""
    P = G.P
    b = np.asarray(beta).reshape(G.M, 2 * P + 1)
    tau = generator(G, jlist)
    n = np.arange(-P, P + 1)
    qidx = (n[None, :] - n[:, None]) + 2 * P
    out = np.einsum("jmnv,mv->jn", tau[:, :, qidx], b)
    return out
