"""Coupling between the inclusions and the layered structure (oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 5 (eqs. repre3_mod, matB, matC):

C maps the outgoing coefficients beta of all inclusions (with their phased near
copies l = -1, 0, 1) to the rows of the empty-structure system: minus the value
and normal derivative on Gamma_1 (the row is u_1 - u_2), plus value and normal
derivative on Gamma_2 (the row is u_2 - u_3), and the middle-layer wall discrepancy, which for a
three-copy source cancels to alpha^2 Phi(L - d) - alpha^{-1} Phi(L + 2d) with Phi
the l = 0 field (and its x-derivative).  All other rows are zero.

B_phys maps the layer unknowns of the middle layer to incoming coefficients at
every inclusion j.  Single and double layers use Graf's addition theorem for
H_0 (P2L):

    (i/4) H_0(k|x - y|) = (i/4) sum_n J_n(k|x - c_j|) e^{in theta(x - c_j)} H_n(k|y - c_j|) e^{-in theta(y - c_j)}

for |x - c_j| < |y - c_j|, and the double layer takes d/dn_y of the same.  The
middle J expansion is re-expanded about c_j (L2L):

    J_q(k|x - c_2|) e^{iq theta(x - c_2)} = sum_n J_{q-n}(k rho) e^{i (q-n) phi} J_n(k|x - c_j|) e^{in theta(x - c_j)},

rho e^{i phi} = c_j - c_2.  (This is the reading used in place of the lemma as
printed in sec. 5, which does not reproduce Graf's theorem.)

Sign convention: A alpha + C beta = f and beta = S (T beta + B_phys alpha); the
paper's B equals -B_phys.

TE polarisation: the flux rows of C take (1/eps_2) d/dn and B_phys's single- and
double-layer parts carry the middle layer's eps_2 (see oracle/layered.py).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .common import outgoing, incoming, grad_wave


def _particle_field_block(G, tx, ty, tdir, images):
    """[n_t, M*nb]: field (or derivative along tdir: scalars or per-target arrays)
    of unit multipoles beta_m[n].

    images: list of (shift_x, weight) pairs applied to the inclusion copies.
    """
    P, M = G.P, G.M
    n = np.arange(-P, P + 1)[None, None, :]
    out = np.zeros((len(tx), M, 2 * P + 1), complex)
    if tdir is not None:
        tdir = tuple(np.broadcast_to(np.asarray(t, float), (len(tx),))[:, None, None]
                     for t in tdir)
    for sx, w in images:
        vx = (tx[:, None] - G.cx[None, :] - sx)[:, :, None]
        vy = (ty[:, None] - G.cy[None, :])[:, :, None]
        if tdir is None:
            f = outgoing(n, G.k2, vx, vy)
        else:
            gx, gy = grad_wave(outgoing, n, G.k2, vx, vy)
            f = gx * tdir[0] + gy * tdir[1]
        out += w * f
    return out.reshape(len(tx), -1)


def assemble_C(G):
    """Dense C of size [n_rows, M(2P+1)]."""
    C = np.zeros((G.n_rows, G.n_beta), complex)
    R = G.row
    three = [(l * G.d, G.alpha ** l) for l in (-1, 0, 1)]
    xg = G.xg
    for line, sgn, rv, rn in ((0, -1.0, "g1v", "g1n"), (1, 1.0, "g2v", "g2n")):
        yt = G.gy[line]
        C[R[rv]] = sgn * _particle_field_block(G, xg, yt, None, three)
        # flux rows: d/dn (times 1/eps_2 for TE: the inclusions sit in the middle layer)
        C[R[rn]] = sgn * G.fl[1] * _particle_field_block(G, xg, yt, G.gn[line], three)
    yw = G.yw[1]
    for rr, tdir in (("w2v", None), ("w2d", (1.0, 0.0))):
        blk = 0
        for xt, wt in ((-1.5 * G.d, G.alpha ** 2), (1.5 * G.d, -G.alpha ** -1)):
            blk = blk + wt * _particle_field_block(G, np.full_like(yw, xt), yw, tdir, [(0.0, 1.0)])
        C[R[rr]] = blk
    return C


def assemble_Bphys(G):
    """Dense B_phys of size [M(2P+1), n_alpha] (nonzero on mu1, sig1, mu2, sig2, a2)."""
    P, M = G.P, G.M
    nb = 2 * P + 1
    B = np.zeros((M, nb, G.n_alpha), complex)
    n = np.arange(-P, P + 1)[None, :, None]
    k = G.k2
    for line, cm, cs in ((0, "mu1", "sig1"), (1, "mu2", "sig2")):
        S = 0
        D = 0
        nx, ny = (v[None, None, :] for v in G.gn[line])
        for l in (-1, 0, 1):
            vx = (G.xg[None, :] + l * G.d - G.cx[:, None])[:, None, :]
            vy = (G.gy[line][None, :] - G.cy[:, None])[:, None, :] + 0 * vx
            # H_n(k|v|) e^{-in theta_v} = (-1)^n F_{-n}(v); the double layer takes its
            # derivative along the source normal
            sgn = (-1.0) ** np.abs(n)
            S = S + G.alpha ** l * sgn * outgoing(-n, k, vx, vy)
            gx, gy = grad_wave(outgoing, -n, k, vx, vy)
            D = D + G.alpha ** l * sgn * (nx * gx + ny * gy)
        # arc-length weights; the middle layer's potentials carry eps_2 for TE
        w = G.gw[line][None, None, :]
        B[:, :, G.col[cs]] = G.pv[1] * 0.25j * w * S
        B[:, :, G.col[cm]] = G.pv[1] * 0.25j * w * D
    Q2 = G.Q[1]
    q = np.arange(-Q2, Q2 + 1)[None, None, :]
    cx2, cy2 = G.jc[1]
    vx = (G.cx - cx2)[:, None, None]
    vy = (G.cy - cy2)[:, None, None]
    B[:, :, G.col["a2"]] = incoming(q - n, k, vx, vy)
    return B.reshape(M * nb, G.n_alpha)
