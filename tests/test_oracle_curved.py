"""Pins of the oracle's curved interfaces (graphs y = +-h + sum_m a_m cos(2 pi m x/d)
+ b_m sin(2 pi m x/d); paper secs. 3 and 6).

Each pin is fixed independently of the oracle's curved-interface code:
  * the locally corrected rule for the four same-interface kernel differences
    (weighted S and D, N, T) on a curved graph against 30-digit adaptive
    quadrature (mpmath) of the kernels written out from their definitions, on a
    smooth windowed density;
  * the empty curved slab against the Rayleigh method (plane-wave expansions in each
    layer matched at collocation points on both interfaces; valid for these small
    amplitudes), TM and TE;
  * equal indices: the curved interfaces are invisible (no reflection, the incident
    wave transmitted unchanged);
  * a grating with inclusions between curved interfaces conserves energy flux and
    its Bragg amplitudes follow the structure under a shift along x by x0
    (c_n -> c_n e^{-2 pi i n x0 / d}); LU = GMRES.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.layered import curve_kernel_limits, curve_kernels
from oracle.quadrature import correction_weights
from oracle.solver import Reduced
from paper_1412_7466_amd import inputs

PROFILES = [inputs.interface_profile((), (0.05,), (0.04,), (0.02,)),
            inputs.interface_profile((0.02, 0.01), (0.03,), (), (0.03, 0.01))]


# --- the local rule on a curved graph ---------------------------------------------

def _graph(x, q=0, m=np):
    """y = 0.1 sin(2 pi x) + 0.05 cos(4 pi x) and its derivatives."""
    w1, w2 = 2 * m.pi, 4 * m.pi
    if q == 0:
        return 0.1 * m.sin(w1 * x) + 0.05 * m.cos(w2 * x)
    if q == 1:
        return 0.1 * w1 * m.cos(w1 * x) - 0.05 * w2 * m.sin(w2 * x)
    return -0.1 * w1 ** 2 * m.sin(w1 * x) - 0.05 * w2 ** 2 * m.cos(w2 * x)


def test_local_rule_on_a_curved_graph():
    s, a, hs, K = 0.13, 0.45, 1.0 / 512, 6
    ka, kb, wa, wb, kap = 12.0, 18.0, 2.25, 4.0, 3.0

    def dens(t, m=np):
        u = (t - s) / a
        w = m.exp(1 - 1 / (1 - u * u)) if abs(u) < 1 else 0
        return m.exp(1j * kap * t) * (1 + 0.3 * m.cos(2 * m.pi * t)) * w

    def normal(t, m=np):
        d1 = _graph(t, 1, m)
        sp_ = m.sqrt(1 + d1 * d1)
        return (-d1 / sp_, 1 / sp_), sp_

    # corrected trapezoid rule on the nodes s + j hs
    J = int(a / hs)
    j = np.arange(-J, J + 1)
    t = s + j * hs
    g = np.array([dens(v) for v in t])
    ns, sps = normal(s)
    nt, spt = normal(t)
    ctr = j == 0
    kv = curve_kernels(ka, kb, wa, wb, np.where(ctr, 1.0, s - t), _graph(s) - _graph(t), ns,
                       nt, spt)
    lim = curve_kernel_limits(ka, kb, wa, wb, sps, _graph(s, 2))
    p = np.arange(-K, K + 1)
    rule = {}
    for q in ("S", "D", "N", "T"):
        kern, phi = kv[q]
        w = correction_weights(np.where(p == 0, lim[q][0], phi[J + p]), lim[q][0], lim[q][1],
                               hs, K)
        rule[q] = hs * np.sum(np.where(ctr, 0, kern) * g) + np.sum(w * g[J + p])

    # adaptive quadrature of the kernels from their definitions, 30 digits
    mp.mp.dps = 30
    cache = {}

    def kernels(tt):
        if tt in cache:
            return cache[tt]
        ms = mp.mpf(s)
        Rx, Ry = ms - tt, _graph(ms, 0, mp) - _graph(tt, 0, mp)
        r = mp.sqrt(Rx * Rx + Ry * Ry)
        (sx, sy), _ = normal(ms, mp)
        (tx, ty), spd = normal(tt, mp)
        Rs, Rt, nn = Rx * sx + Ry * sy, Rx * tx + Ry * ty, sx * tx + sy * ty
        H = {(k, n): mp.mpc(0, 0.25) * mp.hankel1(n, k * r) for k in (ka, kb) for n in (0, 1, 2)}
        out = {"S": (wa * H[ka, 0] - wb * H[kb, 0]) * spd,
               "D": (wa * ka * H[ka, 1] - wb * kb * H[kb, 1]) * Rt / r * spd,
               "N": -(ka * H[ka, 1] - kb * H[kb, 1]) * Rs / r * spd,
               "T": ((ka * H[ka, 1] - kb * H[kb, 1]) * nn / r
                     - (ka ** 2 * H[ka, 2] - kb ** 2 * H[kb, 2]) * Rs * Rt / r ** 2) * spd}
        cache[tt] = out
        return out

    delta = mp.mpf("1e-10")
    for q in ("S", "D", "N", "T"):
        fn = lambda tt: kernels(tt)[q] * dens(tt, mp)
        ref = mp.quad(fn, [s - a, s - delta]) + mp.quad(fn, [s + delta, s + a])
        # the omitted 2 delta around the target, to leading order (a 1e-9 part)
        ref += 2 * delta * (lim[q][0] * (mp.log(delta) - 1) + lim[q][1]) * dens(mp.mpf(s), mp)
        scale = max(1.0, abs(rule[q]))
        assert abs(complex(ref) - rule[q]) < 1e-12 * scale, q


# --- the empty curved slab against the Rayleigh method ----------------------------

def _rayleigh(pb, Nr, te):
    """Rayleigh-Bloch expansions in each layer (layer 2 both ways) matched at
    4(2 Nr + 1) points on each interface in the least-squares sense; returns the
    orders and the reflected / transmitted amplitudes on Gamma_u / Gamma_d."""
    d, h = pb.d, pb.h
    k = [pb.omega * n for n in pb.n_layer]
    eps = [n ** 2 for n in pb.n_layer] if te else [1.0, 1.0, 1.0]
    kap = k[0] * math.sin(pb.phi)
    n = np.arange(-Nr, Nr + 1)
    kn = kap + 2 * np.pi * n / d

    def beta(kk):
        v = kk ** 2 - kn ** 2
        return np.where(v >= 0, np.sqrt(np.abs(v)) + 0j, 1j * np.sqrt(np.abs(v)))

    b1, b2, b3 = beta(k[0]), beta(k[1]), beta(k[2])
    Q = 4 * len(n)
    x = -d / 2 + (np.arange(Q) + 0.5) * d / Q

    def prof(j, q):
        out = np.full_like(x, (h if j == 0 else -h) if q == 0 else 0.0)
        a, b = pb.interface[j]
        for m in range(1, len(a) + 1):
            w = 2 * np.pi * m / d
            c, s = np.cos(w * x), np.sin(w * x)
            out = out + (a[m - 1] * (c, -s)[q] + b[m - 1] * (s, c)[q]) * w ** q
        return out

    E = np.exp(1j * np.outer(x, kn))
    nb = len(n)
    Mx = np.zeros((4 * Q, 4 * nb), complex)
    rhs = np.zeros(4 * Q, complex)

    def wave(bet, y, yref, sgn, slope):
        # e^{i kn x + i sgn bet (y - yref)} and its derivative along (-f', 1)
        w = E * np.exp(1j * sgn * bet[None, :] * (y - yref)[:, None])
        return w, 1j * (-slope[:, None] * kn[None, :] + sgn * bet[None, :]) * w

    # unknowns: r (layer 1 up, referred to y = h), A (layer 2 up, to -h),
    # B (layer 2 down, to h), t (layer 3 down, to -h)
    for top in (True, False):
        y, sl = prof(0 if top else 1, 0), prof(0 if top else 1, 1)
        r0 = 0 if top else 2 * Q
        wA, dA = wave(b2, y, -h, 1, sl)
        wB, dB = wave(b2, y, h, -1, sl)
        if top:
            wr, dr = wave(b1, y, h, 1, sl)
            Mx[r0:r0 + Q, :nb] = wr
            Mx[r0 + Q:r0 + 2 * Q, :nb] = dr / eps[0]
            sgn = -1.0
        else:
            wt, dt = wave(b3, y, -h, -1, sl)
            Mx[r0:r0 + Q, 3 * nb:] = -wt
            Mx[r0 + Q:r0 + 2 * Q, 3 * nb:] = -dt / eps[2]
            sgn = 1.0
        Mx[r0:r0 + Q, nb:2 * nb] = sgn * wA
        Mx[r0:r0 + Q, 2 * nb:3 * nb] = sgn * wB
        Mx[r0 + Q:r0 + 2 * Q, nb:2 * nb] = sgn * dA / eps[1]
        Mx[r0 + Q:r0 + 2 * Q, 2 * nb:3 * nb] = sgn * dB / eps[1]
        if top:
            k1c = k[0] * math.cos(pb.phi)
            ui = np.exp(1j * (kap * x - k1c * y))
            rhs[:Q] = -ui
            rhs[Q:2 * Q] = -1j * (-sl * kap - k1c) * ui / eps[0]
    sol = np.linalg.lstsq(Mx, rhs, rcond=None)[0]
    y0 = pb.disc.y0
    return n, sol[:nb] * np.exp(1j * b1 * (y0 - h)), sol[3 * nb:] * np.exp(1j * b3 * (y0 - h))


@pytest.mark.parametrize("te", [False, True])
@pytest.mark.parametrize("prof", [0, 1])
def test_curved_slab_matches_rayleigh_method(te, prof):
    pb = inputs.empty_slab(omega=10.0, h=0.5, interface=PROFILES[prof])
    if te:
        pb.polarization = "TE"
    out = Reduced(pb).bragg(np.zeros(0))
    n, r, t = _rayleigh(pb, 25, te)
    orders = list(out["orders"])
    err = 0.0
    for i, nn in enumerate(n):
        if nn in orders:
            j = orders.index(nn)
            err = max(err, abs(out["c"][j] - r[i]), abs(out["d"][j] - t[i]))
    assert err < 1e-9
    assert out["flux_err"] < 1e-10
    # the interfaces' shape matters at this level
    flat = Reduced(inputs.empty_slab(omega=10.0, h=0.5)).bragg(np.zeros(0))
    i0 = orders.index(0)
    assert abs(flat["c"][i0] - out["c"][i0]) > 1e-3


def test_equal_indices_make_curved_interfaces_invisible():
    pb = inputs.empty_slab(omega=10.0, h=0.5, n_layer=(1.5, 1.5, 1.5), interface=PROFILES[1])
    red = Reduced(pb)
    out = red.bragg(np.zeros(0))
    i0 = list(out["orders"]).index(0)
    k = pb.omega * 1.5
    d0 = np.exp(1j * k * math.cos(pb.phi) * pb.disc.y0)
    assert np.max(np.abs(out["c"])) < 1e-10
    assert abs(out["d"][i0] - d0) < 1e-10
    assert np.max(np.abs(np.delete(out["d"], i0))) < 1e-10


# --- inclusions between curved interfaces ------------------------------------------

@pytest.mark.parametrize("te", [False, True])
def test_curved_grating_flux_and_solvers(te):
    pb = inputs.curved(12, 6, seed=21)
    if te:
        pb.polarization = "TE"
    red = Reduced(pb)
    b_lu = red.solve_lu()
    out = red.bragg(b_lu)
    assert out["flux_err"] < 1e-10
    b_gm = red.solve_gmres(tol=1e-13)
    assert np.linalg.norm(red.D * (b_gm - b_lu)) < 1e-11 * np.linalg.norm(red.D * b_lu)


def test_curved_grating_shift_along_x():
    pb = inputs.curved(8, 6, seed=5)
    x0 = 0.1234
    sh = inputs.curved(8, 6, seed=5)
    a, b = pb.interface[:, 0, :], pb.interface[:, 1, :]
    m = np.arange(1, a.shape[1] + 1)[None, :]
    w = 2 * np.pi * m * x0 / pb.d
    sh.interface = np.stack([a * np.cos(w) - b * np.sin(w), a * np.sin(w) + b * np.cos(w)],
                            axis=1)
    sh.x = (pb.x + x0 + pb.d / 2) % pb.d - pb.d / 2
    o1 = Reduced(pb).bragg(Reduced(pb).solve_lu())
    red2 = Reduced(sh)
    o2 = red2.bragg(red2.solve_lu())
    ph = np.exp(-2j * np.pi * o1["orders"] * x0 / pb.d)
    sel = o1["prop1"] | o1["prop3"]
    assert np.max(np.abs(o2["c"] - o1["c"] * ph)[o1["prop1"]]) < 1e-9
    assert np.max(np.abs(o2["d"] - o1["d"] * ph)[o1["prop3"]]) < 1e-9
    assert sel.any()
