"""Pseudo-inverse, reduced operator, direct and iterative solves, outputs (oracle).

Test infrastructure only (see oracle/__init__.py).

Paper sec. 5 (eqs. finalsys, applypA, schur and the preconditioned system):
with A alpha + C beta = f and beta = S (T beta + B_phys alpha), eliminating
alpha = A^+ (f - C beta) gives

    K beta = (I - S T + S B_phys A^+ C) beta = S B_phys A^+ f,

the paper's (I - S T - S B A^+ C) beta = -S B A^+ f with B = -B_phys.
A^+ g = V Sigma^+ (U^* g) from the SVD of A (never formed explicitly).  Readings:
columns of A are equilibrated to unit 2-norm first; Sigma^+ keeps 1/sigma_j for
sigma_j >= eps * sigma_1 and drops the rest ("truncate"); the literal cap
min(1/sigma_j, 1/eps) is available as rule="cap".

Reading (scaling): the paper does not discuss the scaling of the multipole basis.
With the orders P used here the outgoing coefficients of small disks span dozens
of decades and K itself is numerically singular, so the system is solved in the
basis normalised by each multipole's size on its own disk boundary: with
D = diag(|H_|n|(k_2 R_m)|), GMRES (and LU) run on D K D^{-1} (D beta) = D b and
beta = D^{-1} (D beta).  This is a diagonal similarity: the exact solution is
unchanged, and the stopping test is the relative residual of the normalised
system.

Outputs (sec. 2, sec. 6): the Rayleigh-Bloch coefficients c_n, d_n are the last
two blocks of alpha = A^+ (f - C beta); for propagating orders
R_n = k_{1,n} |c_n|^2 / (k_1 cos phi), T_n = k_{3,n} |d_n|^2 / (k_1 cos phi), and the
flux error is |sum R_n + sum T_n - 1| (lossless media).
"""
from __future__ import annotations

import time

import numpy as np
import scipy.linalg as sla
import scipy.special as sp

from .common import Geometry
from .layered import assemble_A, rhs_f
from .multiple import mie_coefficients, dense_T, TranslationTable
from .coupling import assemble_C, assemble_Bphys
from .inclusion import scattering_matrix


class PseudoInverse:
    """A^+ via the SVD of the column-equilibrated A."""

    def __init__(self, A, eps=1e-10, rule="truncate"):
        cn = np.linalg.norm(A, axis=0)
        cn = np.where(cn > 0, cn, 1.0)
        self.E = 1.0 / cn
        U, s, Vh = np.linalg.svd(A * self.E[None, :], full_matrices=False)
        self.U, self.s, self.Vh = U, s, Vh
        if rule == "truncate":
            sp_ = np.where(s >= eps * s[0], 1.0 / np.where(s > 0, s, 1.0), 0.0)
        elif rule == "cap":
            sp_ = np.minimum(1.0 / np.where(s > 0, s, np.inf), 1.0 / eps)
        else:
            raise ValueError(rule)
        self.splus = sp_
        self.rank = int(np.count_nonzero(sp_))

    def apply(self, g):
        g = np.asarray(g)
        t = self.U.conj().T @ g
        if g.ndim == 1:
            return self.E * (self.Vh.conj().T @ (self.splus * t))
        return self.E[:, None] * (self.Vh.conj().T @ (self.splus[:, None] * t))


class Reduced:
    """The reduced inclusion system of one Problem, built in FP64 on the CPU."""

    def __init__(self, pb, dense=None, pinv_rule="truncate", verbose=False):
        t0 = time.perf_counter()
        self.G = G = Geometry(pb)
        self.A = assemble_A(G)
        self.f = rhs_f(G)
        self.pinv = PseudoInverse(self.A, pb.disc.pinv_eps, pinv_rule)
        # single-inclusion scattering matrices (sec. 4.1): the Mie diagonal s of a disk,
        # or, for the non-circular inclusions of eq. par1, a dense (2P+1)^2 block per
        # inclusion from its boundary integral equation (self.S, [M][2P+1][2P+1])
        self.S = None
        if getattr(pb, "shape", None) is not None and G.M and G.te:
            raise NotImplementedError("non-circular inclusions are written for TM")
        if getattr(pb, "shape", None) is not None and G.M and G.lossy:
            raise NotImplementedError("non-circular inclusions are written lossless")
        if getattr(pb, "shape", None) is not None and G.M:
            sh = np.asarray(pb.shape, float)
            self.S = np.stack([scattering_matrix(a1, a2, a3, rot, G.k2, kp, G.P,
                                                 n=pb.shape_nodes // 2)
                               for (a1, a2, a3, rot), kp in zip(sh, G.kp)])
            self.s = None
        else:
            te = dict(eps2=G.eps[1], epsp=G.eps_incl) if G.te else {}
            self.s = (mie_coefficients(G.k2, G.kp, G.rad, G.P, **te).reshape(-1) if G.M
                      else np.zeros(0))
        n = np.abs(np.arange(-G.P, G.P + 1))
        self.D = (np.abs(sp.hankel1(n[None, :], G.k2 * G.rad[:, None])).reshape(-1)
                  if G.M else np.zeros(0))
        if dense is None:
            dense = G.n_beta <= 4000
        self.dense = dense
        if G.M:
            self.C = assemble_C(G)
            self.B = assemble_Bphys(G)
            if dense:
                self.T = dense_T(G)
            else:
                self.table = TranslationTable(G)
        self.setup_seconds = time.perf_counter() - t0
        if verbose:
            print(f"oracle setup {self.setup_seconds:.1f}s  A {self.A.shape} rank {self.pinv.rank}")

    # -- operator pieces -------------------------------------------------
    def T_apply(self, x):
        return self.T @ x if self.dense else self.table.apply(x)

    def lowrank_apply(self, x):
        """B_phys A^+ C x (the incoming field of the layers due to x)."""
        return self.B @ self.pinv.apply(self.C @ x)

    def S_mul(self, v):
        """The block-diagonal scattering matrix times v (a vector or [n, cols])."""
        if self.S is None:
            return self.s * v if v.ndim == 1 else self.s[:, None] * v
        M, nb = self.G.M, self.G.nb
        if v.ndim == 1:
            return np.einsum("mln,mn->ml", self.S, v.reshape(M, nb)).reshape(-1)
        return np.einsum("mln,mnc->mlc", self.S, v.reshape(M, nb, -1)).reshape(M * nb, -1)

    def K_apply(self, x):
        return x - self.S_mul(self.T_apply(x) - self.lowrank_apply(x))

    def rhs(self):
        return self.S_mul(self.B @ self.pinv.apply(self.f))

    def K_dense(self):
        n = self.G.n_beta
        W = self.pinv.apply(self.C)       # [n_alpha, n]
        return np.eye(n) - self.S_mul(self.T - self.B @ W)

    # -- solves ------------------------------------------------------------
    def solve_lu(self):
        """LU of the normalised system D K D^{-1} (D beta) = D b."""
        D = self.D
        Kh = D[:, None] * self.K_dense() / D[None, :]
        return sla.lu_solve(sla.lu_factor(Kh), D * self.rhs()) / D

    def solve_gmres(self, tol=1e-11, maxit=2000, x0=None, restart=None):
        """GMRES on the normalised system; tol is its relative residual."""
        D = self.D
        xh0 = None if x0 is None else D * x0
        bh, it, res = gmres(lambda v: D * self.K_apply(v / D), D * self.rhs(), tol=tol,
                            maxit=maxit, x0=xh0, restart=restart)
        self.gmres_iters, self.gmres_resid = it, res
        return bh / D

    def solve_full_ls(self):
        """Least squares of the whole system [[A, C], [-S B_phys, I - S T]] (small only).

        The inclusion rows are multiplied by S (the left preconditioner), so the
        system is [[A, C], [-S B_phys, I - S T]] [alpha; beta] = [f; 0]; columns are
        equilibrated and the same singular-value cut is applied.
        """
        G = self.G
        n = G.n_beta
        D = self.D
        # beta columns in normalised units (D beta), inclusion rows scaled by D
        top = np.hstack([self.A, self.C / D[None, :]])
        bot = np.hstack([-D[:, None] * self.S_mul(self.B),
                         D[:, None] * (np.eye(n) - self.S_mul(self.T)) / D[None, :]])
        F = np.vstack([top, bot])
        rhs = np.concatenate([self.f, np.zeros(n, complex)])
        pi = PseudoInverse(F, self.G.pb.disc.pinv_eps)
        sol = pi.apply(rhs)
        return sol[G.n_alpha:] / D, sol[:G.n_alpha]

    # -- outputs -------------------------------------------------------------
    def alpha_vec(self, beta):
        g = self.f - (self.C @ beta if self.G.M else 0)
        return self.pinv.apply(g)

    def absorbed(self, beta):
        """Fraction of the incident energy flux absorbed by the (disk) inclusions.

        Around disk m the field is sum_n (a_n J_n + b_n H_n) e^{in theta} with b = beta_m
        and incoming a_n = b_n / s_n; its outward energy flux through a circle is
        4 sum_n (|b_n|^2 + Re(conj(a_n) b_n)) (Wronskian J Y' - J' Y = 2 / (pi z)), so the
        disk absorbs -4 sum_n |b_n|^2 (|s_n|^2 + Re s_n) / |s_n|^2 (zero for lossless
        disks: |1 + 2 s_n| = 1).  Normalised by the incident flux d k_1 cos(phi) of one
        period (TE: the flux densities carry 1/eps of their medium)."""
        G = self.G
        if not G.M or not G.lossy:
            return 0.0
        s = self.s
        b = np.asarray(beta)
        nz = np.abs(s) > 0
        per = np.where(nz, np.abs(b) ** 2 * (np.abs(s) ** 2 + s.real) / np.where(nz, np.abs(s) ** 2, 1), 0)
        w = G.eps[0] / G.eps[1] if G.te else 1.0
        return float(-4.0 * w * per.sum() / (G.d * G.k1 * G.cosphi))

    def bragg(self, beta):
        """Propagating orders, c_n, d_n, R_n, T_n, the absorbed fraction and the flux
        (energy balance) error |sum R + sum T + absorbed - 1|."""
        G = self.G
        al = self.alpha_vec(beta)
        c = al[G.col["c"]]
        d = al[G.col["d"]]
        prop1 = (np.abs(G.k1n.imag) == 0) & (G.k1n.real > 0)
        inc = G.k1 * G.cosphi
        Rn = np.where(prop1, G.k1n.real * np.abs(c) ** 2 / inc, 0.0)
        ab = self.absorbed(beta) if G.M else 0.0
        if G.lossy3:
            # absorbing substrate: order n of the Rayleigh-Bloch expansion below
            # Gamma_d carries the downward flux Re(k_3n) |d_n|^2 across Gamma_d (no
            # cross terms: the kappa_n differ by multiples of 2 pi / d).  The layer
            # also absorbs between Gamma_2 and Gamma_d, including the evanescent near
            # field of inclusions close to the interface, which the amplitudes at
            # Gamma_d no longer resolve; so R + T + A < 1 and flux_err is NaN.
            # "Propagating" marks the orders with Re(k_3^2 - kappa_n^2) > 0.
            # TE: the flux of a wave is Re(k_y / eps) |amplitude|^2, over k_1 cos(phi) / eps_1
            prop3 = (G.k3 ** 2 - G.kapn ** 2).real > 0
            Tn = ((G.eps[0] * G.k3n / G.eps[2]).real if G.te else G.k3n.real) * np.abs(d) ** 2 / inc
            flux = float("nan")
        else:
            prop3 = (np.abs(G.k3n.imag) == 0) & (G.k3n.real > 0)
            # TE: the energy flux of a wave is (k_y / eps) |amplitude|^2
            t3 = G.eps[0] / G.eps[2] if G.te else 1.0
            Tn = np.where(prop3, t3 * G.k3n.real * np.abs(d) ** 2 / inc, 0.0)
            flux = abs(Rn.sum() + Tn.sum() + ab - 1.0)
        return dict(orders=G.rb, c=c, d=d, R=Rn, T=Tn, prop1=prop1, prop3=prop3,
                    flux_err=flux, absorbed=ab)


def gmres(Aop, b, tol=1e-11, maxit=2000, x0=None, restart=None):
    """Restarted GMRES with modified Gram-Schmidt (Saad & Schultz), FP64.

    Stops when ||b - A x|| / ||b|| <= tol (the "GMRES error" of the paper's tables).
    Returns (x, iterations, final relative residual).
    """
    n = b.shape[0]
    restart = restart or min(maxit, 400)
    x = np.zeros(n, complex) if x0 is None else np.array(x0, complex)
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0, 0.0
    total = 0
    while True:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol or total >= maxit:
            return x, total, beta / bn
        V = np.zeros((restart + 1, n), complex)
        H = np.zeros((restart + 1, restart), complex)
        V[0] = r / beta
        g = np.zeros(restart + 1, complex)
        g[0] = beta
        cs = np.zeros(restart, complex)
        sn = np.zeros(restart, complex)
        j_done = 0
        for j in range(restart):
            w = Aop(V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den else 1.0
            sn[j] = bb / den if den else 0.0
            H[j, j] = den
            H[j + 1, j] = 0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            total += 1
            j_done = j + 1
            if abs(g[j + 1]) / bn <= tol or total >= maxit:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x = x + V[:j_done].T @ y
