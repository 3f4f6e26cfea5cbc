"""Zeta-corrected trapezoid rule for log-singular kernels on a flat line (oracle).

Test infrastructure only (see oracle/__init__.py).

The paper discretizes the layer potentials by Nystrom with a locally corrected
trapezoid rule (sec. 3, "Alpert quadrature corrections"; the Alpert tables are
not printed).  On a flat interface the same-line kernels that survive are the
differences S_{k_a} - S_{k_b} and T_{k_a} - T_{k_b}; each has the form
K(s) = phi(s) ln|s| + psi(s) with smooth phi, psi.  For equispaced nodes s_j = j h
around a target at s_0 = 0 the punctured trapezoid sum has the generalized
Euler-Maclaurin expansion (Navot):

  int K tau ds = h sum_{j != 0} K(jh) tau(jh)
                 + h [psi(0) + phi(0) ln(h / 2 pi)] tau(0)
                 + sum_{k=1}^{Kz} 2 zeta'(-2k) h^{2k+1} (phi tau)^{(2k)}(0) / (2k)!
                 + O(h^{2 Kz + 1}),

with 2 zeta'(-2k) / (2k)! = (-1)^k zeta(2k+1) / (2 pi)^{2k}.  The even
derivatives of phi*tau are taken by centred finite differences on the
(2 Kz + 1)-point stencil around the target.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def fd_weights(z, m):
    """Finite-difference weights at 0 for derivatives 0..m on nodes z.

    Fornberg's recursion (Math. Comp. 51, 1988).  Returns c[q, j] so that
    f^{(q)}(0) ~ sum_j c[q, j] f(z_j).
    """
    z = np.asarray(z, float)
    n = len(z)
    c = np.zeros((m + 1, n))
    c1 = 1.0
    c4 = z[0]
    c[0, 0] = 1.0
    for i in range(1, n):
        mn = min(i, m)
        c2 = 1.0
        c5 = c4
        c4 = z[i]
        for j in range(i):
            c3 = z[i] - z[j]
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k, i] = c1 * (k * c[k - 1, i - 1] - c5 * c[k, i - 1]) / c2
                c[0, i] = -c1 * c5 * c[0, i - 1] / c2
            for k in range(mn, 0, -1):
                c[k, j] = (c4 * c[k, j] - k * c[k - 1, j]) / c3
            c[0, j] = c4 * c[0, j] / c3
        c1 = c2
    return c


def zeta_coefficients(K):
    """2 zeta'(-2k) / (2k)! for k = 1..K, via the functional equation."""
    k = np.arange(1, K + 1)
    return (-1.0) ** k * sp.zeta(2 * k + 1, 1) / (2 * np.pi) ** (2 * k)


def correction_weights(phi_vals, phi0, psi0, h, K):
    """Stencil weights (offsets -K..K) that correct the punctured trapezoid sum.

    phi_vals: phi(p h) for p = -K..K (the p = 0 entry is phi(0)).
    Returns w[p + K] such that the corrected rule is
        h sum_{j != 0} K(jh) tau_j + sum_p w[p + K] tau_p.
    """
    p = np.arange(-K, K + 1)
    c = fd_weights(p.astype(float), 2 * K)
    zc = zeta_coefficients(K)
    w = np.zeros(2 * K + 1, dtype=complex)
    for kk in range(1, K + 1):
        w += h * zc[kk - 1] * c[2 * kk] * phi_vals
    w[K] += h * (psi0 + phi0 * np.log(h / (2 * np.pi)))
    return w
