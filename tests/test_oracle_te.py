"""Pins of the oracle's TE polarisation (u = H_z: u and (1/eps) du/dn continuous,
eps = n^2; the paper treats TM only and names TE as an extension).

Each pin is fixed by physics or a closed form, independently of the oracle's TE
factors: the empty slab against the TE transfer-matrix (Fresnel) solution; the TE
Mie coefficients against energy (|1 + 2 s_n| = 1) and the TE interface conditions at
r = R; in a transparent background the Bragg amplitudes are the plane-wave expansion
of the phased multipole array (the TE flux scaling of C and A must cancel); a
grating with inclusions conserves the TE energy flux; LU, GMRES and the full least
squares agree; TE and TM differ where the indices differ.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from paper_1412_7466_amd import inputs
from oracle.multiple import mie_coefficients
from oracle.solver import Reduced

WOOD = math.asin((2 * math.pi - 10.0) / 10.0)


def _te(pb):
    pb.polarization = "TE"
    return pb


def _fresnel_te(pb):
    """TE transfer matrix of the flat three-layer slab: u continuous and
    (1/eps) du/dy continuous at y = +-h."""
    n1, n2, n3 = pb.n_layer
    e1, e2, e3 = n1 ** 2, n2 ** 2, n3 ** 2
    k1, k2, k3 = (pb.omega * n for n in pb.n_layer)
    kap = k1 * math.sin(pb.phi)
    k1y = k1 * math.cos(pb.phi)
    k2y = np.sqrt(k2 ** 2 - kap ** 2 + 0j)
    k3y = np.sqrt(k3 ** 2 - kap ** 2 + 0j)
    h = pb.h
    E = np.exp
    M = np.array([[E(1j * k1y * h), -E(1j * k2y * h), -E(-1j * k2y * h), 0],
                  [1j * k1y / e1 * E(1j * k1y * h), -1j * k2y / e2 * E(1j * k2y * h),
                   1j * k2y / e2 * E(-1j * k2y * h), 0],
                  [0, E(-1j * k2y * h), E(1j * k2y * h), -E(1j * k3y * h)],
                  [0, 1j * k2y / e2 * E(-1j * k2y * h), -1j * k2y / e2 * E(1j * k2y * h),
                   1j * k3y / e3 * E(1j * k3y * h)]])
    rhs = np.array([-E(-1j * k1y * h), 1j * k1y / e1 * E(-1j * k1y * h), 0, 0])
    r, _, _, t = np.linalg.solve(M, rhs)
    y0 = pb.disc.y0
    return r * E(1j * k1y * y0), t * E(1j * k3y * y0)


@pytest.mark.parametrize("phi", [-math.pi / 5, 0.3, WOOD])
def test_empty_slab_is_te_fresnel(phi):
    pb = _te(inputs.empty_slab(phi=phi))
    red = Reduced(pb)
    out = red.bragg(np.zeros(0))
    c0, d0 = _fresnel_te(pb)
    i0 = list(red.G.rb).index(0)
    assert abs(out["c"][i0] - c0) < 1e-12
    assert abs(out["d"][i0] - d0) < 1e-12
    others = np.delete(np.arange(len(out["c"])), i0)
    # evanescent orders: leakage of the order of the pseudo-inverse cut (1e-10)
    assert np.max(np.abs(out["c"][others])) < 5e-11
    assert np.max(np.abs(out["d"][others])) < 5e-11
    p1 = out["prop1"].copy()
    p1[i0] = False
    p3 = out["prop3"].copy()
    p3[i0] = False
    assert np.max(np.abs(out["c"][p1]), initial=0) < 1e-12
    assert np.max(np.abs(out["d"][p3]), initial=0) < 1e-12
    assert out["flux_err"] < 1e-12
    # and differs from TM at this contrast
    tm = Reduced(inputs.empty_slab(phi=phi)).bragg(np.zeros(0))
    assert abs(tm["c"][i0] - out["c"][i0]) > 1e-3


def test_te_mie_energy_and_interface():
    k2, n2, npp, R, P = 15.0, 1.5, 2.5, 0.04, 8
    om = k2 / n2
    kp = om * npp
    s = mie_coefficients(k2, np.array([kp]), np.array([R]), P, eps2=n2 ** 2,
                         epsp=np.array([npp ** 2])).reshape(-1)
    assert np.max(np.abs(np.abs(1 + 2 * s) - 1)) < 1e-13
    # interface conditions for J_n + s_n H_n outside and gamma_n J_n(kp r) inside
    n = np.arange(-P, P + 1)
    out_v = sp.jv(n, k2 * R) + s * sp.hankel1(n, k2 * R)
    out_d = k2 * (sp.jvp(n, k2 * R) + s * sp.h1vp(n, k2 * R)) / n2 ** 2
    gam = out_v / sp.jv(n, kp * R)
    in_d = kp * gam * sp.jvp(n, kp * R) / npp ** 2
    assert np.max(np.abs(in_d - out_d) / np.abs(out_d)) < 1e-12
    # TM coefficients are different at this contrast
    stm = mie_coefficients(k2, np.array([kp]), np.array([R]), P).reshape(-1)
    assert np.max(np.abs(stm - s)) > 1e-3


def test_te_transparent_background_plane_wave_expansion():
    """Equal media: alpha = A^+(-C beta) must give the plane-wave expansion of the
    phased multipole array, whatever the polarisation's eps factors."""
    pb = _te(inputs.small(5, 8, seed=11, n_layer=(1.5, 1.5, 1.5)))
    red = Reduced(pb)
    G = red.G
    rng = np.random.default_rng(2)
    nu = np.arange(-G.P, G.P + 1)
    beta = (rng.standard_normal((G.M, len(nu))) + 1j * rng.standard_normal((G.M, len(nu))))
    beta *= 0.3 ** np.abs(nu)[None, :]
    al = red.pinv.apply(-red.C @ beta.reshape(-1))
    c = al[G.col["c"]]
    d = al[G.col["d"]]
    k = G.k2
    kn = G.k1n
    kap = G.kapn
    up = ((kn - 1j * kap) / k)[:, None] ** nu[None, :]
    dn = ((-(kn + 1j * kap)) / k)[:, None] ** nu[None, :]
    y0 = G.y0
    c_ref = np.zeros_like(c)
    d_ref = np.zeros_like(d)
    for m in range(G.M):
        ex = np.exp(-1j * kap * G.cx[m])
        c_ref += 2 / (G.d * kn) * ex * np.exp(1j * kn * (y0 - G.cy[m])) * (up @ beta[m])
        d_ref += 2 / (G.d * kn) * ex * np.exp(1j * kn * (y0 + G.cy[m])) * (dn @ beta[m])
    sel = np.abs(G.rb - G.rb[len(G.rb) // 2]) <= 6
    assert np.max(np.abs(c - c_ref)[sel]) < 1e-10 * np.max(np.abs(c_ref))
    assert np.max(np.abs(d - d_ref)[sel]) < 1e-10 * np.max(np.abs(d_ref))


@pytest.mark.parametrize("M,P,seed", [(4, 10, 1), (12, 6, 21)])
def test_te_flux_and_solvers(M, P, seed):
    pb = _te(inputs.tiny_m4() if M == 4 else inputs.small(M, P, seed=seed))
    red = Reduced(pb)
    b_lu = red.solve_lu()
    out = red.bragg(b_lu)
    assert out["flux_err"] < 1e-10
    b_gm = red.solve_gmres(tol=1e-13)
    assert np.linalg.norm(red.D * (b_gm - b_lu)) < 1e-11 * np.linalg.norm(red.D * b_lu)
    b_ls, _ = red.solve_full_ls()
    assert np.linalg.norm(red.D * (b_ls - b_lu)) < 1e-9 * np.linalg.norm(red.D * b_lu)
    # the TM solution of the same geometry is different
    tm = Reduced(inputs.tiny_m4() if M == 4 else inputs.small(M, P, seed=seed)).solve_lu()
    assert np.linalg.norm(red.D * (tm - b_lu)) > 1e-3 * np.linalg.norm(red.D * b_lu)
