"""Pins of the oracle's absorbing substrate: the bottom layer's index n_3 + i n3_im
(the paper names complex permittivities as an extension, sec. 7; TM and TE).

Each pin is fixed independently of the oracle's layer assembly: the empty flat slab
against the transfer-matrix (Fresnel) solution with the complex k_3, and its energy
balance (reflected power plus the power of the transmitted wave at the interface, which
the substrate absorbs, equal the incident power); with disks in the middle layer, the
reflected powers and the disks' coefficients do not depend on where the artificial line
Gamma_d is put (a different discretization of the substrate's part of the unit cell);
LU, GMRES and the full least squares agree; the loss changes the solution; the same
for TE, whose substrate factors eps_3 = (n_3 + i n3_im)^2 are complex.  The Bragg
output reports no energy balance here (flux_err NaN): the substrate absorbs above
Gamma_d too.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from oracle.solver import Reduced


def _substrate(pb, n3_im):
    pb.n3_im = n3_im
    return pb


def _fresnel_tm(pb):
    """TM transfer matrix of the flat three-layer slab with k_3 = omega (n_3 + i n3_im):
    u and du/dy continuous at y = +-h; r, t referred to the lines y = +-y0."""
    n1, n2, n3 = pb.n_layer
    k1, k2 = pb.omega * n1, pb.omega * n2
    k3 = pb.omega * (n3 + 1j * pb.n3_im)
    kap = k1 * math.sin(pb.phi)
    k1y = k1 * math.cos(pb.phi)
    k2y = np.sqrt(k2 ** 2 - kap ** 2 + 0j)
    k3y = np.sqrt(k3 ** 2 - kap ** 2)       # principal root: Re, Im > 0
    assert k3y.real > 0 and k3y.imag > 0
    h = pb.h
    E = np.exp
    M = np.array([[E(1j * k1y * h), -E(1j * k2y * h), -E(-1j * k2y * h), 0],
                  [1j * k1y * E(1j * k1y * h), -1j * k2y * E(1j * k2y * h),
                   1j * k2y * E(-1j * k2y * h), 0],
                  [0, E(-1j * k2y * h), E(1j * k2y * h), -E(1j * k3y * h)],
                  [0, 1j * k2y * E(-1j * k2y * h), -1j * k2y * E(1j * k2y * h),
                   1j * k3y * E(1j * k3y * h)]])
    rhs = np.array([-E(-1j * k1y * h), 1j * k1y * E(-1j * k1y * h), 0, 0])
    r, _, _, t = np.linalg.solve(M, rhs)
    y0 = pb.disc.y0
    return r * E(1j * k1y * y0), t * E(1j * k3y * y0)


@pytest.mark.parametrize("phi,n3_im", [(-math.pi / 5, 0.05), (0.3, 0.12)])
def test_empty_slab_is_fresnel(phi, n3_im):
    pb = _substrate(inputs.empty_slab(phi=phi), n3_im)
    red = Reduced(pb)
    out = red.bragg(np.zeros(0))
    c0, d0 = _fresnel_tm(pb)
    i0 = list(red.G.rb).index(0)
    assert abs(out["c"][i0] - c0) < 1e-12
    assert abs(out["d"][i0] - d0) < 1e-12
    others = np.delete(np.arange(len(out["c"])), i0)
    assert np.max(np.abs(out["c"][others])) < 5e-11
    assert np.max(np.abs(out["d"][others])) < 5e-11
    # the loss is felt: the lossless slab reflects differently
    lossless = Reduced(inputs.empty_slab(phi=phi)).bragg(np.zeros(0))
    assert abs(lossless["c"][i0] - out["c"][i0]) > 1e-3
    assert math.isnan(out["flux_err"])
    # energy: the plane wave t e^{-i k3y (y + y0)} carries Re(k3y) |t|^2 e^{2 Im(k3y)(y0 - h)}
    # across the interface y = -h; with the reflected power it makes the incident one
    k1y = pb.omega * pb.n_layer[0] * math.cos(phi)
    k3y = np.sqrt((pb.omega * (pb.n_layer[2] + 1j * n3_im)) ** 2
                  - (pb.omega * pb.n_layer[0] * math.sin(phi)) ** 2)
    t_iface = k3y.real * abs(out["d"][i0]) ** 2 * math.exp(2 * k3y.imag * (pb.disc.y0 - pb.h))
    assert abs(out["R"][i0] + t_iface / k1y - 1.0) < 1e-12
    assert out["T"][i0] < t_iface / k1y   # the strip above Gamma_d absorbs
    assert abs(out["T"][i0] - k3y.real * abs(out["d"][i0]) ** 2 / k1y) < 1e-15


def test_powers_do_not_depend_on_gamma_d():
    pb = _substrate(inputs.small(10, 6, seed=5), 0.06)
    pb2 = _substrate(inputs.small(10, 6, seed=5), 0.06)
    pb2.disc = dataclasses.replace(pb.disc, y0=pb.disc.y0 * 1.12)
    o1 = Reduced(pb).bragg(Reduced(pb).solve_lu())
    red2 = Reduced(pb2)
    b2 = red2.solve_lu()
    o2 = red2.bragg(b2)
    assert np.max(np.abs(o1["R"] - o2["R"])) < 1e-9
    # the transmitted powers at the lower line are smaller by what the longer strip absorbs
    assert o2["T"].sum() < o1["T"].sum()
    red1 = Reduced(pb)
    b1 = red1.solve_lu()
    D = red1.D
    assert np.linalg.norm(D * (b1 - b2)) < 1e-8 * np.linalg.norm(D * b1)


def test_solvers_agree_and_loss_matters():
    pb = _substrate(inputs.small(12, 6, seed=21), 0.08)
    red = Reduced(pb)
    b_lu = red.solve_lu()
    b_gm = red.solve_gmres(tol=1e-13)
    assert np.linalg.norm(red.D * (b_gm - b_lu)) < 1e-11 * np.linalg.norm(red.D * b_lu)
    b_ls, _ = red.solve_full_ls()
    assert np.linalg.norm(red.D * (b_ls - b_lu)) < 1e-9 * np.linalg.norm(red.D * b_lu)
    b0 = Reduced(inputs.small(12, 6, seed=21)).solve_lu()
    assert np.linalg.norm(red.D * (b0 - b_lu)) > 1e-3 * np.linalg.norm(red.D * b_lu)


def test_curved_powers_do_not_depend_on_gamma_d():
    """Curved Gamma_2 over the substrate: its same-interface blocks take the kernel
    differences and zeta corrections at the complex k_3 (ln(k_3/2) complex); moving
    Gamma_d must leave the reflected powers and the disks' coefficients unchanged."""
    pb = inputs.lossy_substrate(8, 6, seed=32, n3_im=0.06, curved_iface=True)
    pb2 = inputs.lossy_substrate(8, 6, seed=32, n3_im=0.06, curved_iface=True)
    pb2.disc = dataclasses.replace(pb.disc, y0=pb.disc.y0 * 1.1)
    red1, red2 = Reduced(pb), Reduced(pb2)
    b1, b2 = red1.solve_lu(), red2.solve_lu()
    o1, o2 = red1.bragg(b1), red2.bragg(b2)
    assert np.max(np.abs(o1["R"] - o2["R"])) < 1e-9
    D = red1.D
    assert np.linalg.norm(D * (b1 - b2)) < 1e-8 * np.linalg.norm(D * b1)


@pytest.mark.parametrize("curved", [False, True])
def test_balance_not_reported(curved):
    """With disks (absorbing or not, flat or curved interfaces) R + T + A stays
    below 1 by what the substrate absorbs above Gamma_d, and flux_err is NaN."""
    pb = inputs.lossy_substrate(8, 6, seed=32, n3_im=0.05, curved_iface=curved)
    red = Reduced(pb)
    out = red.bragg(red.solve_lu())
    assert math.isnan(out["flux_err"])
    tot = out["R"].sum() + out["T"].sum() + out["absorbed"]
    assert 0.0 < 1.0 - tot < 0.5


def _fresnel_te(pb):
    """TE transfer matrix with eps_3 = (n_3 + i n3_im)^2: u and (1/eps) du/dy
    continuous at y = +-h."""
    n1, n2, n3 = pb.n_layer
    n3c = n3 + 1j * pb.n3_im
    e1, e2, e3 = n1 ** 2, n2 ** 2, n3c ** 2
    k1, k2, k3 = pb.omega * n1, pb.omega * n2, pb.omega * n3c
    kap = k1 * math.sin(pb.phi)
    k1y = k1 * math.cos(pb.phi)
    k2y = np.sqrt(k2 ** 2 - kap ** 2 + 0j)
    k3y = np.sqrt(k3 ** 2 - kap ** 2)
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
    return r * E(1j * k1y * y0), t * E(1j * k3y * y0), k3y, e1, e3


@pytest.mark.parametrize("phi,n3_im", [(-math.pi / 5, 0.05), (0.3, 0.12)])
def test_te_empty_slab_is_fresnel(phi, n3_im):
    """TE over the absorbing substrate: the layer factors eps_3 and 1/eps_3 of the
    substrate's potentials and flux rows are complex."""
    pb = _substrate(inputs.empty_slab(phi=phi), n3_im)
    pb.polarization = "TE"
    red = Reduced(pb)
    out = red.bragg(np.zeros(0))
    c0, d0, k3y, e1, e3 = _fresnel_te(pb)
    i0 = list(red.G.rb).index(0)
    assert abs(out["c"][i0] - c0) < 1e-12
    assert abs(out["d"][i0] - d0) < 1e-12
    others = np.delete(np.arange(len(out["c"])), i0)
    assert np.max(np.abs(out["c"][others])) < 5e-11
    assert np.max(np.abs(out["d"][others])) < 5e-11
    # energy: the TE flux of a wave is Re(k_y / eps) |u|^2; at the interface the
    # transmitted wave carries Re(k3y / eps_3) |d0|^2 e^{2 Im(k3y)(y0 - h)}
    k1y = pb.omega * pb.n_layer[0] * math.cos(phi)
    t_iface = (k3y / e3).real * abs(d0) ** 2 * math.exp(2 * k3y.imag * (pb.disc.y0 - pb.h))
    assert abs(out["R"][i0] + t_iface / (k1y / e1) - 1.0) < 1e-12
    assert abs(out["T"][i0] - e1 * (k3y / e3).real * abs(out["d"][i0]) ** 2 / k1y) < 1e-15
    # TE differs from TM over the same substrate
    tm = Reduced(_substrate(inputs.empty_slab(phi=phi), n3_im)).bragg(np.zeros(0))
    assert abs(tm["c"][i0] - out["c"][i0]) > 1e-3


def test_te_powers_do_not_depend_on_gamma_d():
    pb = _substrate(inputs.small(10, 6, seed=5), 0.06)
    pb2 = _substrate(inputs.small(10, 6, seed=5), 0.06)
    pb.polarization = pb2.polarization = "TE"
    pb2.disc = dataclasses.replace(pb.disc, y0=pb.disc.y0 * 1.12)
    red1, red2 = Reduced(pb), Reduced(pb2)
    b1, b2 = red1.solve_lu(), red2.solve_lu()
    o1, o2 = red1.bragg(b1), red2.bragg(b2)
    assert np.max(np.abs(o1["R"] - o2["R"])) < 1e-9
    D = red1.D
    assert np.linalg.norm(D * (b1 - b2)) < 1e-8 * np.linalg.norm(D * b1)
