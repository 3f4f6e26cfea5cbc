"""Derived quantities, discretization nodes and multipole helpers (oracle).

Test infrastructure only (see oracle/__init__.py).

Conventions (paper sec. 2): time dependence e^{-i omega t}; wavenumber k_j =
omega * n_j (mu = 1, eps = n^2); Bloch phase alpha = e^{i kappa d}; Rayleigh-Bloch
wavenumbers kappa_n = kappa + 2 pi n / d and k_{j,n} = sqrt(k_j^2 - kappa_n^2)
taken with non-negative real or imaginary part (eq. rad1/rad2).  The incidence
angle phi is measured from the downward normal: kappa = k_1 sin(phi), and the
incident wave is exp(i (kappa x - k_1 cos(phi) y)) in the top layer only.

Outgoing multipole of order n about c: H_n(k |x-c|) e^{i n theta(x-c)}.
Incoming (local) term: J_n(k |x-c|) e^{i n theta(x-c)}.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def sqrt_branch(v):
    """sqrt(v) for real v, non-negative real part or positive imaginary part.  For
    v with positive imaginary part (an absorbing layer: k^2 - kappa_n^2 with Im k > 0)
    the principal root, whose real and imaginary parts are both positive: each
    Rayleigh-Bloch wave then carries energy away from the layers and decays."""
    v = np.asarray(v)
    if np.iscomplexobj(v) and np.any(v.imag != 0):
        if np.any(v.imag < 0):
            raise ValueError("the layer index must have a non-negative imaginary part")
        return np.sqrt(v.astype(complex))
    v = np.asarray(v.real if np.iscomplexobj(v) else v, dtype=float)
    out = np.where(v >= 0, np.sqrt(np.abs(v)) + 0j, 1j * np.sqrt(np.abs(v)))
    return out


def outgoing(n, k, vx, vy):
    """H_n(k r) e^{i n theta} at displacement (vx, vy); broadcasts over n."""
    r = np.hypot(vx, vy)
    th = np.arctan2(vy, vx)
    return sp.hankel1(n, k * r) * np.exp(1j * n * th)


def incoming(n, k, vx, vy):
    """J_n(k r) e^{i n theta} at displacement (vx, vy); broadcasts over n."""
    r = np.hypot(vx, vy)
    th = np.arctan2(vy, vx)
    return sp.jv(n, k * r) * np.exp(1j * n * th)


def grad_wave(fun, n, k, vx, vy):
    """(d/dx, d/dy) of Z_n(k r) e^{i n theta} for Z in {J, H}.

    From (d_x + i d_y) Z_n e^{in theta} = -k Z_{n+1} e^{i(n+1) theta} and
    (d_x - i d_y) Z_n e^{in theta} = k Z_{n-1} e^{i(n-1) theta}.
    """
    fm = fun(n - 1, k, vx, vy)
    fp = fun(n + 1, k, vx, vy)
    return 0.5 * k * (fm - fp), 0.5j * k * (fm + fp)


class Geometry:
    """All derived quantities of one Problem (geometry + one incidence)."""

    def __init__(self, pb):
        self.pb = pb
        dd = pb.disc
        self.d, self.h = float(pb.d), float(pb.h)
        self.k1, self.k2, self.k3 = (pb.omega * n for n in pb.n_layer)
        # absorbing substrate: k_3 = omega (n_3 + i n3_im), Im k_3 > 0 (sec. 7 names
        # complex permittivities as an extension); for TE its eps_3 = (n_3 + i n3_im)^2
        n3_im = float(getattr(pb, "n3_im", 0.0) or 0.0)
        self.lossy3 = n3_im != 0.0
        if self.lossy3:
            if n3_im < 0:
                raise ValueError("n3_im must be non-negative")
            self.k3 = pb.omega * (pb.n_layer[2] + 1j * n3_im)
        self.kl = (self.k1, self.k2, self.k3)
        self.P = int(pb.P)
        self.M = int(len(pb.x))
        self.cx = np.asarray(pb.x, float)
        self.cy = np.asarray(pb.y, float)
        self.rad = np.asarray(pb.radius, float)
        # inclusion wavenumbers: complex for absorbing inclusions (index n + i n_im)
        n_im = getattr(pb, "n_incl_im", None)
        self.lossy = n_im is not None
        n_p = np.asarray(pb.n_incl, float) + (1j * np.asarray(n_im, float) if self.lossy else 0)
        self.kp = pb.omega * n_p
        # polarisation: TM (u = E_z, u and du/dn continuous) or TE (u = H_z, u and
        # (1/eps) du/dn continuous, eps = n^2).  For TE each layer's potentials carry
        # the factor pv = eps of their layer and the flux rows the factor 1/eps of the
        # layer whose field they take (so the hypersingular parts still cancel); TM
        # has both factors 1.
        self.te = getattr(pb, "polarization", "TM") == "TE"
        self.eps = tuple(n ** 2 for n in pb.n_layer)
        if self.lossy3:  # complex permittivity of the absorbing substrate
            self.eps = (self.eps[0], self.eps[1], (pb.n_layer[2] + 1j * n3_im) ** 2)
        self.eps_incl = n_p ** 2
        self.pv = self.eps if self.te else (1.0, 1.0, 1.0)
        self.fl = tuple(1.0 / e for e in self.eps) if self.te else (1.0, 1.0, 1.0)
        self.kappa = self.k1 * np.sin(pb.phi)
        self.alpha = np.exp(1j * self.kappa * self.d)
        self.cosphi = np.cos(pb.phi)
        # Rayleigh-Bloch orders (eq. rad1/rad2)
        self.rb = dd.n_rb_lo + np.arange(dd.Nrb)
        self.kapn = self.kappa + 2 * np.pi * self.rb / self.d
        self.k1n = sqrt_branch(self.k1 ** 2 - self.kapn ** 2)
        self.k3n = sqrt_branch(self.k3 ** 2 - self.kapn ** 2)
        # interface nodes: cell-centred, equispaced in x (the graphs' parameter),
        # trapezoid weight d/N per unit of x
        N = dd.N
        self.N = N
        self.hs = self.d / N
        self.xg = -self.d / 2 + (np.arange(N) + 0.5) * self.hs
        self.y0 = float(dd.y0)
        # interfaces y = f_j(x) (paper secs. 3, 6): flat at +-h, or graphs of period d
        # with Fourier deviations; at the nodes their heights gy, unit normals gn
        # (pointing up, (-f', 1) / |(1, f')|), speeds sp = |(1, f')| and second
        # derivatives f'', and the arc-length weights gw = hs sp
        iface = getattr(pb, "interface", None)
        self.curved = iface is not None
        self.iface = (np.zeros((2, 2, 0)) if iface is None
                      else np.asarray(iface, float).reshape(2, 2, -1))
        self.gy, self.gn, self.sp, self.gd2, self.gw = [], [], [], [], []
        for j in range(2):
            f0, f1, f2 = (self.f(j, self.xg, q) for q in range(3))
            sp_ = np.sqrt(1.0 + f1 ** 2)
            self.gy.append(f0)
            self.gn.append((-f1 / sp_, 1.0 / sp_))
            self.sp.append(sp_)
            self.gd2.append(f2)
            self.gw.append(self.hs * sp_)
        # wall nodes: Gauss-Legendre on each layer's wall (the walls end on the
        # interfaces at x = +-d/2)
        e1 = float(self.f(0, np.array([self.d / 2]))[0])
        e2 = float(self.f(1, np.array([self.d / 2]))[0])
        spans = ((e1, self.y0), (e2, e1), (-self.y0, e2))
        self.yw = []
        for Nw, (a, b) in zip(dd.Nw, spans):
            t, _ = np.polynomial.legendre.leggauss(Nw)
            self.yw.append(0.5 * (a + b) + 0.5 * (b - a) * t)
        # Gamma_u / Gamma_d nodes
        self.xu = -self.d / 2 + (np.arange(dd.Nu) + 0.5) * self.d / dd.Nu
        # J expansion centres of layers 1, 2, 3 and their orders
        yc = 0.5 * (self.h + self.y0)
        self.jc = ((0.0, yc), (0.0, 0.0), (0.0, -yc))
        self.Q = tuple(int(q) for q in dd.Q)
        # column layout of the empty-structure unknowns
        sizes = [("mu1", N), ("sig1", N), ("mu2", N), ("sig2", N),
                 ("a2", 2 * self.Q[1] + 1), ("a1", 2 * self.Q[0] + 1),
                 ("a3", 2 * self.Q[2] + 1), ("c", dd.Nrb), ("d", dd.Nrb)]
        self.col = {}
        o = 0
        for nm, s in sizes:
            self.col[nm] = slice(o, o + s)
            o += s
        self.n_alpha = o
        # row layout of the conditions
        rs = [("g1v", N), ("g1n", N), ("g2v", N), ("g2n", N),
              ("w2v", dd.Nw[1]), ("w2d", dd.Nw[1]),
              ("w1v", dd.Nw[0]), ("w1d", dd.Nw[0]),
              ("w3v", dd.Nw[2]), ("w3d", dd.Nw[2]),
              ("uv", dd.Nu), ("un", dd.Nu), ("dv", dd.Nu), ("dn", dd.Nu)]
        self.row = {}
        o = 0
        for nm, s in rs:
            self.row[nm] = slice(o, o + s)
            o += s
        self.n_rows = o
        self.nb = 2 * self.P + 1
        self.n_beta = self.M * self.nb

    def f(self, j, x, q=0):
        """q-th x-derivative of interface j's height function at the points x."""
        x = np.asarray(x, float)
        out = np.full_like(x, (self.h if j == 0 else -self.h) if q == 0 else 0.0)
        a, b = self.iface[j]
        for m in range(1, len(a) + 1):
            w = 2 * np.pi * m / self.d
            c, s = np.cos(w * x), np.sin(w * x)
            # d^q/dx^q of a cos(w x) + b sin(w x)
            dc = (c, -s, -c)[q] * w ** q
            ds = (s, c, -s)[q] * w ** q
            out = out + a[m - 1] * dc + b[m - 1] * ds
        return out

    def u_inc(self, x, y):
        """Incident plane wave (top layer only)."""
        return np.exp(1j * (self.kappa * x - self.k1 * self.cosphi * y))
