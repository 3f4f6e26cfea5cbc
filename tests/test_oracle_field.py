"""Pins of the oracle's coupling blocks and of the whole discrete solution, through
the field it represents (oracle/field.py), plus truncation convergence and the
pseudo-inverse rule.

Each test names the passage of the paper it follows.  None of them compares the
oracle with itself: the field is summed from the representation formulas with its
own near-line quadrature (no kernel splitting, no zeta correction, jump relations
not imposed), and the physical conditions the method imposes only at nodes are
checked at points between them.
"""
import dataclasses

import numpy as np
import pytest
import scipy.special as sp

from paper_1412_7466_amd import inputs
from oracle.common import Geometry, incoming
from oracle.coupling import assemble_Bphys
from oracle.field import Field, _jexp, _kernels
from oracle.solver import Reduced

X_OFF = np.array([-0.4321, -0.1, 0.0123, 0.2777, 0.49])   # between interface nodes


@pytest.fixture(scope="module")
def tiny_fine():
    """The M=4 problem with the singular-value cut at 1e-12 (the field's continuity
    between nodes is limited by that cut, see test_pinv_rule_and_eps_sweep)."""
    pb = inputs.tiny_m4(pinv_eps=1e-12)
    red = Reduced(pb)
    beta = red.solve_lu()
    return red, beta, Field(red, beta)


# --- B_phys by Graf's theorem (sec. 5, eq. matB; the L2L reading R13) ---------------

@pytest.mark.parametrize("part", ["sig1", "mu1", "sig2", "mu2", "a2"])
def test_bphys_graf_direct(part):
    """alpha^L = B_phys w is the local (J) expansion about each disk of the field that
    w produces: the three copies of the discretized single or double layer on Gamma_1
    or Gamma_2 (P2L), or the middle J expansion about c_2 (L2L), summed directly at
    points near each centre."""
    pb = inputs.small(5, 12, seed=3)
    G = Geometry(pb)
    B = assemble_Bphys(G)
    nb = 2 * G.P + 1
    n = np.arange(-G.P, G.P + 1)
    rng = np.random.default_rng(4)
    sl = G.col[part]
    k = sl.stop - sl.start
    v = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    if part == "a2":
        v /= (1 + np.abs(np.arange(-G.Q[1], G.Q[1] + 1))) ** 2
    w = np.zeros(G.n_alpha, complex)
    w[sl] = v
    alL = (B @ w).reshape(G.M, nb)
    for j in range(G.M):
        th = np.linspace(0, 2 * np.pi, 7, endpoint=False) + 0.3
        tx = G.cx[j] + 0.1 * G.rad[j] * np.cos(th)
        ty = G.cy[j] + 0.1 * G.rad[j] * np.sin(th)
        if part == "a2":
            direct = _jexp(G, 1, v, tx, ty)[0]
        else:
            ys = G.h if part.endswith("1") else -G.h
            direct = np.zeros(len(tx), complex)
            for l in (-1, 0, 1):
                xs = G.xg[None, :] + l * G.d
                g, _, _, dd, _, _ = _kernels(G.k2, tx[:, None] - xs, ty[:, None] - ys)
                dens = g if part.startswith("sig") else dd
                direct += G.alpha ** l * G.hs * (dens @ v)
        local = incoming(n[None, :], G.k2, (tx - G.cx[j])[:, None],
                         (ty - G.cy[j])[:, None]) @ alL[j]
        assert np.max(np.abs(local - direct)) < 1e-13 * np.max(np.abs(direct)), (part, j)


# --- the whole solution, between the nodes (sec. 2 eqs. bound1-bound3) -----------------

def test_field_quasi_periodic_on_walls(tiny_fine):
    """u(d/2, y) = alpha u(-d/2, y) and the same for u_x, at wall points between the
    Gauss-Legendre nodes, in all three layers (total field)."""
    red, beta, F = tiny_fine
    G = red.G
    for j, (a, b) in enumerate(((G.h, G.y0), (-G.h, G.h), (-G.y0, -G.h))):
        ys = a + (b - a) * np.array([0.17, 0.33, 0.5, 0.71, 0.86])
        uL = F.layer(j, np.full_like(ys, -G.d / 2), ys)
        uR = F.layer(j, np.full_like(ys, G.d / 2), ys)
        assert np.max(np.abs(uR[0] - G.alpha * uL[0])) < 1e-10 * np.max(np.abs(uL[0])), j
        assert np.max(np.abs(uR[1] - G.alpha * uL[1])) < 1e-10 * np.max(np.abs(uL[1])), j


def test_field_continuous_across_interfaces(tiny_fine):
    """Total field and its y-derivative agree from both sides of Gamma_1 (top layer
    with the incident wave vs middle layer) and Gamma_2 at points between the
    interface nodes; each one-sided limit is extrapolated from 8 distances."""
    red, beta, F = tiny_fine
    G = red.G
    for ja, jb, yl in ((0, 1, G.h), (1, 2, -G.h)):
        A = F.limit_on_line(ja, X_OFF, yl, +1)
        B = F.limit_on_line(jb, X_OFF, yl, -1)
        assert np.max(np.abs(A[0] - B[0])) < 1e-11 * np.max(np.abs(A[0])), yl
        assert np.max(np.abs(A[2] - B[2])) < 1e-10 * np.max(np.abs(A[2])), yl


def test_field_matches_rayleigh_bloch_lines(tiny_fine):
    """On Gamma_u and Gamma_d the layer representation equals the Rayleigh-Bloch
    expansion with the computed c_n, d_n (value and y-derivative), between nodes."""
    red, beta, F = tiny_fine
    G = red.G
    xs = np.array([-0.37, 0.011, 0.29])
    for top, j, y in ((True, 0, G.y0), (False, 2, -G.y0)):
        r = F.rayleigh(top, xs, np.full_like(xs, y))
        lay = F.layer(j, xs, np.full_like(xs, y), total=False)
        assert np.max(np.abs(r[0] - lay[0])) < 1e-10 * np.max(np.abs(r[0])), top
        assert np.max(np.abs(r[2] - lay[2])) < 1e-10 * np.max(np.abs(r[2])), top


@pytest.mark.parametrize("which", ["tiny", "small12"])
def test_field_inclusions_scatter_their_incoming_field(which):
    """beta_m = S_m alpha_m (sec. 4.1, 5): the field arriving at disk m (everything in
    the middle layer's representation except m's own multipoles), sampled on a circle
    inside the disk and expanded in J_n(k2 rho) e^{in theta} by FFT, times the Mie
    coefficients, gives back beta_m (normalised by D = |H_|n|(k2 r_m)|)."""
    pb = inputs.tiny_m4() if which == "tiny" else inputs.small(12, 8, seed=9, phi=0.3)
    red = Reduced(pb)
    G = red.G
    beta = red.solve_lu()
    F = Field(red, beta)
    nb = 2 * G.P + 1
    b = beta.reshape(G.M, nb)
    s = red.s.reshape(G.M, nb)
    n = np.arange(-G.P, G.P + 1)
    K = 64
    th = 2 * np.pi * np.arange(K) / K
    for m in range(min(G.M, 4)):
        rho = 0.9 * G.rad[m]
        u_in = F.layer(1, G.cx[m] + rho * np.cos(th), G.cy[m] + rho * np.sin(th),
                       skip=(m, 0))[0]
        c = (np.fft.fft(u_in) / K)[n % K]              # alpha_n J_n(k2 rho)
        pred = s[m] * c / sp.jv(n, G.k2 * rho)
        D = np.abs(sp.hankel1(np.abs(n), G.k2 * G.rad[m]))
        ok = np.abs(c) > 1e-9 * np.abs(c).max()
        assert ok.sum() >= 9
        err = np.abs(D * (pred - b[m]))[ok]
        assert err.max() < 1e-12 * np.abs(D * b[m]).max(), (which, m)


# --- truncation (sec. 6: convergence of the discretization) ----------------------------

def _amps(pb, **kw):
    red = Reduced(pb, **kw)
    o = red.bragg(red.solve_lu())
    return np.concatenate([o["c"][o["prop1"]], o["d"][o["prop3"]]]), o["flux_err"], red


def test_truncation_convergence():
    """Propagating Bragg amplitudes of the M=4 problem converge as the multipole order
    P, the interface node count N and the middle J order Q2 grow (each against the
    default discretization: P=10, N=128, Q2=43)."""
    base = inputs.tiny_m4()
    ref, _, _ = _amps(base)

    def err(pb):
        return np.max(np.abs(_amps(pb)[0] - ref)) / np.max(np.abs(ref))

    eP = [err(dataclasses.replace(base, P=P)) for P in (2, 4, 6)]
    assert eP[0] > 1e-6 and eP[0] > 1e3 * eP[1] > 1e6 * eP[2] and eP[2] < 1e-12, eP
    eN = [err(dataclasses.replace(base, disc=dataclasses.replace(base.disc, N=N)))
          for N in (48, 80, 112)]
    assert eN[0] > eN[1] > eN[2] and eN[2] < 1e-12 and eN[0] < 1e-9, eN
    Q = base.disc.Q
    eQ = [err(dataclasses.replace(base, disc=dataclasses.replace(base.disc, Q=(Q[0], q, Q[2]))))
          for q in (4, 8, 16, 24)]
    assert eQ[0] > 10 * eQ[1] > 100 * eQ[2] and eQ[2] > eQ[3] and eQ[3] < 1e-11, eQ


# --- the pseudo-inverse (sec. 5 eq. applypA, reading R8) --------------------------------

def test_pinv_rule_and_eps_sweep():
    """Truncating (default) or capping (the literal min(1/sigma, 1/eps)) the inverse
    singular values, with eps in {1e-9, 1e-10, 1e-11}: Bragg amplitudes agree with the
    eps = 1e-13 solution to 1e-9 and flux holds to 1e-11; the field's continuity between
    nodes is set by the cut (worse at larger eps), which is why the field pins above use
    eps = 1e-12."""
    base = inputs.tiny_m4()
    ref, _, _ = _amps(dataclasses.replace(base, disc=dataclasses.replace(base.disc,
                                                                         pinv_eps=1e-13)))
    jumps = {}
    for rule in ("truncate", "cap"):
        for eps in (1e-9, 1e-10, 1e-11):
            pb = dataclasses.replace(base, disc=dataclasses.replace(base.disc, pinv_eps=eps))
            a, flux, red = _amps(pb, pinv_rule=rule)
            assert np.max(np.abs(a - ref)) < 1e-9 * np.max(np.abs(ref)), (rule, eps)
            assert flux < 1e-11, (rule, eps)
            if rule == "cap":
                assert red.pinv.rank == red.A.shape[1]
            if eps != 1e-10:
                F = Field(red, red.solve_lu())
                A = F.limit_on_line(0, X_OFF[:2], red.G.h, +1, npts=6)
                B = F.limit_on_line(1, X_OFF[:2], red.G.h, -1, npts=6)
                jumps[(rule, eps)] = np.max(np.abs(A[0] - B[0])) / np.max(np.abs(A[0]))
    for rule in ("truncate", "cap"):
        assert jumps[(rule, 1e-11)] < jumps[(rule, 1e-9)], jumps


def test_field_continuous_across_disk_boundaries(tiny_fine):
    """Inside each disk the field is sum_n gamma_n J_n(k_p r) e^{in theta} (sec. 4.1);
    on the boundary it meets the middle layer's representation in value and radial
    derivative (TM, equal mu), at points between any quadrature nodes."""
    red, beta, F = tiny_fine
    G = red.G
    n = np.arange(-G.P, G.P + 1)
    th = np.linspace(0, 2 * np.pi, 9, endpoint=False) + 0.1
    for m in range(G.M):
        R = G.rad[m]
        tx = G.cx[m] + R * np.cos(th)
        ty = G.cy[m] + R * np.sin(th)
        u, ux, uy = F.layer(1, tx, ty)
        ur = ux * np.cos(th) + uy * np.sin(th)
        e = np.exp(1j * np.outer(th, n))
        kp = G.kp[m]
        u_in = (e * sp.jv(n, kp * R)) @ F.gamma[m]
        ur_in = (e * kp * sp.jvp(n, kp * R)) @ F.gamma[m]
        # the local expansions are truncated at |n| <= P = 10 here, at their outer radius
        assert np.max(np.abs(u_in - u)) < 1e-10 * np.max(np.abs(u)), m
        assert np.max(np.abs(ur_in - ur)) < 1e-9 * np.max(np.abs(ur)), m
        # Field.total picks the interior just inside the boundary
        ins, val = F.inside(G.cx[m] + 0.999 * R * np.cos(th), G.cy[m] + 0.999 * R * np.sin(th))
        assert np.all(ins)
