"""Pins of the oracle's absorbing inclusions (complex refractive index n + i n_im,
n_im > 0; the paper's flux identity holds for real wavenumbers only).

Fixed independently of the oracle's lossy code:
  * the Mie coefficients with a complex interior wavenumber satisfy the interface
    conditions at r = R (SciPy's Bessel functions of complex argument), TM and TE;
    absorbing disks scatter less than they receive, |1 + 2 s_n| < 1;
  * energy balance of a grating with absorbing disks: the reflected and transmitted
    Rayleigh-Bloch fluxes (from the layer unknowns) plus the power absorbed inside the
    disks (from each disk's own incoming and outgoing coefficients) equal the incident
    flux; the absorption is a sizeable fraction;
  * n_im = 0 is the lossless problem; LU = GMRES.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle.multiple import mie_coefficients
from oracle.solver import Reduced
from paper_1412_7466_amd import inputs


@pytest.mark.parametrize("te", [False, True])
def test_lossy_mie_interface_conditions(te):
    k2, n2, P, R = 15.0, 1.5, 10, 0.04
    om = k2 / n2
    npc = np.array([2.5 + 0.3j, 1.8 + 0.05j])
    kp = om * npc
    e2, ep = (n2 ** 2, npc ** 2) if te else (1.0, np.ones(2))
    s = mie_coefficients(k2, kp, np.full(2, R), P,
                         **(dict(eps2=e2, epsp=ep) if te else {}))
    n = np.arange(-P, P + 1)
    for m in range(2):
        out_v = sp.jv(n, k2 * R) + s[m] * sp.hankel1(n, k2 * R)
        out_d = k2 * (sp.jvp(n, k2 * R) + s[m] * sp.h1vp(n, k2 * R)) / e2
        gam = out_v / sp.jv(n, kp[m] * R)
        in_d = kp[m] * gam * sp.jvp(n, kp[m] * R) / ep[m]
        assert np.max(np.abs(in_d - out_d) / np.abs(out_d)) < 1e-12
        # absorbing: |1 + 2 s_n| <= 1, strictly below for |n| <= 2 (the high
        # orders barely reach the interior)
        assert np.all(np.abs(1 + 2 * s[m]) <= 1 + 1e-15)
        assert np.all(np.abs(1 + 2 * s[m][np.abs(n) <= 2]) < 1 - 1e-6)
    s0 = mie_coefficients(k2, np.array([om * 2.5 + 0j]), np.array([R]), P)
    s1 = mie_coefficients(k2, np.array([om * 2.5]), np.array([R]), P)
    assert np.max(np.abs(s0 - s1)) < 1e-15


@pytest.mark.parametrize("te", [False, True])
def test_lossy_energy_balance_and_solvers(te):
    pb = inputs.lossy(12, 8, seed=21)
    if te:
        pb.polarization = "TE"
    red = Reduced(pb)
    b_lu = red.solve_lu()
    out = red.bragg(b_lu)
    assert out["absorbed"] > 0.05
    assert out["flux_err"] < 1e-10        # R + T + absorbed = 1
    assert abs(out["R"].sum() + out["T"].sum() - 1) > 0.05
    b_gm = red.solve_gmres(tol=1e-13)
    assert np.linalg.norm(red.D * (b_gm - b_lu)) < 1e-11 * np.linalg.norm(red.D * b_lu)


def test_zero_loss_is_the_lossless_problem():
    pb = inputs.lossy(8, 6, seed=5)
    pb.n_incl_im = np.zeros(pb.M)
    red = Reduced(pb)
    b = red.solve_lu()
    out = red.bragg(b)
    assert abs(out["absorbed"]) < 1e-12
    ref = Reduced(inputs.small(8, 6, seed=5)).solve_lu()
    assert np.max(np.abs(red.D * (b - ref))) < 1e-13 * np.max(np.abs(red.D * ref))
