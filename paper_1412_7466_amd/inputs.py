"""Seeded synthetic workloads for the layered-grating multi-inclusion problem.

This module only *generates inputs*: geometry (seeded random sequential packing of
disks in the middle layer), the incidence, and the integer sizes of the
discretization.  It holds none of the method's arithmetic (no Green's functions,
no special functions, no linear algebra), so that both the CPU oracle and the
HIP library can consume the same inputs without sharing any code that computes
the answer.

Problem statement (paper section 2): a period-d three-layer TM grating, interfaces
Gamma_1 near y=+h and Gamma_2 near y=-h (flat, or graphs of period d given by
their Fourier coefficients, as in the paper's section 6), refractive indices
n_layer = (top, middle, bottom), M disks of radius r_m and index n_m inside the
middle layer, plane-wave incidence at angle phi measured from the downward
normal (so the horizontal wavenumber is k_1 sin(phi)), multipole order P.

Discretization sizes follow the paper's description of its discretization
(section 3: equispaced interface nodes, Gauss-Legendre wall nodes, J expansions of
2Q+1 terms, Rayleigh-Bloch modes, artificial lines at +-y0) with the concrete
rules of derive_discretization below, where the paper gives no numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Discretization:
    """Integer sizes and positions that fix the discrete problem."""
    N: int                 # nodes on each interface (cell-centred, equispaced)
    Nw: tuple              # Gauss-Legendre nodes on the walls of layers (1, 2, 3)
    Q: tuple               # J-expansion orders of layers (1, 2, 3): 2Q+1 terms each
    Nu: int                # nodes on each of Gamma_u, Gamma_d (cell-centred)
    n_rb_lo: int           # lowest Rayleigh-Bloch order kept
    Nrb: int               # number of Rayleigh-Bloch orders kept (each side)
    y0: float              # Gamma_u at y=+y0, Gamma_d at y=-y0
    zeta_K: int = 6        # zeta-correction stencil half-width (order 2K+1)
    pinv_eps: float = 1e-10  # relative singular-value cut of the pseudo-inverse


@dataclasses.dataclass
class Problem:
    """One geometry + one incidence (one right-hand side)."""
    d: float
    h: float
    n_layer: tuple          # (top, middle, bottom) refractive indices
    omega: float
    phi: float              # incidence angle from the downward normal (rad)
    P: int                  # multipole order, 2P+1 coefficients per inclusion
    x: np.ndarray           # inclusion centres (M,)
    y: np.ndarray
    radius: np.ndarray
    n_incl: np.ndarray
    disc: Discretization
    name: str = ""
    seed: Optional[int] = None
    # non-circular inclusions (paper eq. par1): per inclusion (a1, a2, a3, rot), the
    # boundary rho(t) (cos(t + rot), sin(t + rot)), rho = a1 + a2 cos(a3 t), with
    # radius = a1 + |a2| its enclosing circle; None: disks of the given radii.
    # shape_nodes: boundary nodes of each inclusion's integral equation.
    shape: Optional[np.ndarray] = None
    shape_nodes: int = 64
    # "TM" (the paper's polarisation: u = E_z, u and du/dn continuous) or "TE"
    # (u = H_z: u and (1/eps) du/dn continuous, eps = n^2)
    polarization: str = "TM"
    # curved interfaces (graphs of period d, paper secs. 3 and 6): interface[j] =
    # [[a_1..a_F], [b_1..b_F]] for Gamma_1 (j = 0) and Gamma_2 (j = 1), the graph
    # y = (+h or -h) + sum_m a_m cos(2 pi m x / d) + b_m sin(2 pi m x / d);
    # None: both flat.
    interface: Optional[np.ndarray] = None
    # absorbing inclusions: imaginary parts of the inclusions' refractive indices
    # (n_incl + i n_incl_im, n_incl_im >= 0; the wave e^{i k x} with k = omega n decays);
    # None: lossless
    n_incl_im: Optional[np.ndarray] = None
    # absorbing substrate: imaginary part of the bottom layer's index (n_3 + i n3_im,
    # n3_im >= 0); 0: lossless
    n3_im: float = 0.0

    @property
    def M(self) -> int:
        return int(self.x.shape[0])

    def digest(self) -> str:
        """Short hash of every input value (used to check stored fixtures)."""
        import hashlib
        hsh = hashlib.sha256()
        for v in (self.d, self.h, *self.n_layer, self.omega, self.phi, self.P):
            hsh.update(np.float64(v).tobytes())
        for a in (self.x, self.y, self.radius, self.n_incl):
            hsh.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        dd = self.disc
        hsh.update(np.array([dd.N, *dd.Nw, *dd.Q, dd.Nu, dd.n_rb_lo, dd.Nrb, dd.zeta_K],
                            dtype=np.int64).tobytes())
        hsh.update(np.array([dd.y0, dd.pinv_eps], dtype=np.float64).tobytes())
        if self.shape is not None:
            hsh.update(np.ascontiguousarray(self.shape, dtype=np.float64).tobytes())
            hsh.update(np.int64(self.shape_nodes).tobytes())
        if self.polarization != "TM":
            hsh.update(self.polarization.encode())
        if self.n3_im:
            hsh.update(np.float64(self.n3_im).tobytes())
        if self.n_incl_im is not None:
            hsh.update(b"n_incl_im")
            hsh.update(np.ascontiguousarray(self.n_incl_im, dtype=np.float64).tobytes())
        if self.interface is not None:
            hsh.update(b"interface")
            hsh.update(np.ascontiguousarray(self.interface, dtype=np.float64).tobytes())
        return hsh.hexdigest()[:16]


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def pack_disks(M: int, d: float, h: float, r_lo: float, r_hi: float,
               n_lo: float, n_hi: float, gap: float, seed: int,
               clearance: Optional[float] = None, max_tries: int = 1_000_000):
    """Seeded random sequential packing of M disks in the middle layer.

    Radii are drawn first, then indices, from PCG64(seed).  Disks are placed
    largest first (stable in index order); each try draws x ~ U[-d/2, d/2) and
    y ~ U[-h+c+r, h-c-r] with c = clearance (default max(gap, 0.02)), and is
    accepted when the minimum-image distance (period d in x) to every placed
    disk is at least r_i + r_j + gap.  Returns arrays in the original index
    order.  Raises RuntimeError if a disk cannot be placed.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if r_lo == r_hi:
        radius = np.full(M, float(r_lo))
    else:
        radius = rng.uniform(r_lo, r_hi, size=M)
    if n_lo == n_hi:
        n_incl = np.full(M, float(n_lo))
    else:
        n_incl = rng.uniform(n_lo, n_hi, size=M)
    c = max(gap, 0.02) if clearance is None else clearance
    order = np.argsort(-radius, kind="stable")
    xs = np.empty(M)
    ys = np.empty(M)
    # uniform cell grid over the periodic strip for the overlap checks
    rmax = float(radius.max()) if M else 0.0
    cell = max(2.0 * rmax + gap, 1e-9)
    ncx = max(1, int(d / cell))
    ncy = max(1, int(2 * h / cell))
    cw, chh = d / ncx, 2 * h / ncy
    grid = {}
    placed_r = np.empty(M)
    for cnt, i in enumerate(order):
        r = radius[i]
        ylo, yhi = -h + c + r, h - c - r
        if ylo > yhi:
            raise RuntimeError("disk does not fit between the interfaces")
        for _ in range(max_tries):
            x = rng.uniform(-d / 2, d / 2)
            y = rng.uniform(ylo, yhi)
            gx = int((x + d / 2) / cw) % ncx
            gy = min(ncy - 1, max(0, int((y + h) / chh)))
            ok = True
            for ox in (-1, 0, 1):
                if not ok:
                    break
                for oy in (-1, 0, 1):
                    lst = grid.get(((gx + ox) % ncx, gy + oy))
                    if not lst:
                        continue
                    for k in lst:
                        dx = x - xs[k]
                        dx -= d * math.floor(dx / d + 0.5)
                        dy = y - ys[k]
                        if dx * dx + dy * dy < (r + placed_r[k] + gap) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
            if ok:
                break
        else:
            raise RuntimeError(f"packing failed at disk {cnt} of {M}")
        xs[i], ys[i], placed_r[i] = x, y, r
        grid.setdefault((gx, gy), []).append(i)
        if ncx < 3:  # tiny grids: the neighbour sweep above may alias; keep exact
            pass
    return xs, ys, radius, n_incl


def min_image_gap(x, y, radius, d):
    """Smallest edge-to-edge minimum-image distance between two disks."""
    M = len(x)
    best = np.inf
    for i in range(M):
        dx = x[i] - x[i + 1:]
        dx -= d * np.floor(dx / d + 0.5)
        dy = y[i] - y[i + 1:]
        g = np.sqrt(dx * dx + dy * dy) - radius[i] - radius[i + 1:]
        if g.size:
            best = min(best, float(g.min()))
    return best


# ----------------------------------------------------------------------------
# discretization sizes
# ----------------------------------------------------------------------------

def _round_up(v: int, m: int) -> int:
    return ((v + m - 1) // m) * m


def derive_discretization(d, h, n_layer, omega, phi, y_incl, P,
                          zeta_K=6, pinv_eps=1e-10, N_min=120, amp=0.0) -> Discretization:
    """Sizes of the discrete problem from the geometry and the frequency.

    * y0 = h + d/2; J centres at the middle of each truncated layer.
    * amp bounds how far a curved interface leaves y = +-h (0 for flat ones); the
      layers' extents below grow by it.
    * N = max(N_min, ceil(6 d / d_c), ceil(8 k_max d / pi)) rounded up to a
      multiple of 16; d_c is the smallest inclusion-centre-to-interface distance.
    * Q_j = max(ceil(k_j R_j + 15), ceil(ln(1e-14) / ln(R_j / D_j))) with R_j the
      largest distance from the J centre to a point of the layer's cell and D_j
      the distance to the nearest source copy two or more periods away.
    * Nw_j = max(ceil(k_j H_j / 2) + 24, ceil(0.8 (2 Q_j + 1))) Gauss-Legendre
      nodes per wall, H_j the wall height.
    * Rayleigh-Bloch orders: the 2*nh+1 orders centred on -round(kappa d / 2pi),
      nh = max(20, ceil(k_max d / 2pi) + 12).
    * Nu = max(50, ceil(1.25 Nrb)).
    """
    k = [omega * n for n in n_layer]
    kmax = max(k)
    y0 = h + d / 2
    hu = (y0 - h) / 2  # half height of the top / bottom truncated layers
    if len(y_incl):
        hc = h - amp
        dc = float(np.min(np.minimum(hc - np.asarray(y_incl), np.asarray(y_incl) + hc)))
        n_dc = math.ceil(6 * d / dc)
    else:
        n_dc = 0
    N = _round_up(max(N_min, n_dc, math.ceil(8 * kmax * d / math.pi)), 16)
    # layer 1 (top) and 3 (bottom) share the geometry; layer 2 is the middle
    R1 = math.hypot(d / 2, hu + amp)
    D1 = math.hypot(1.5 * d, max(hu - amp, 0.0))
    R2 = math.hypot(d / 2, h + amp)
    D2 = 1.5 * d
    Qs = []
    for kj, R, D in ((k[0], R1, D1), (k[1], R2, D2), (k[2], R1, D1)):
        Qs.append(max(math.ceil(kj * R + 15), math.ceil(math.log(1e-14) / math.log(R / D))))
    H = (y0 - h + amp, 2 * (h + amp), y0 - h + amp)
    Nw = tuple(max(math.ceil(kj * Hj / 2) + 24, math.ceil(0.8 * (2 * Qj + 1)))
               for kj, Hj, Qj in zip(k, H, Qs))
    kappa = k[0] * math.sin(phi)
    nc = -int(round(kappa * d / (2 * math.pi)))
    nh = max(20, math.ceil(kmax * d / (2 * math.pi)) + 12)
    Nrb = 2 * nh + 1
    Nu = max(50, math.ceil(1.25 * Nrb))
    return Discretization(N=N, Nw=Nw, Q=tuple(Qs), Nu=Nu, n_rb_lo=nc - nh, Nrb=Nrb,
                          y0=y0, zeta_K=zeta_K, pinv_eps=pinv_eps)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

STACK = (1.0, 1.5, 2.0)


def interface_profile(g1_cos=(), g1_sin=(), g2_cos=(), g2_sin=()) -> np.ndarray:
    """The interface array of a Problem, [2][2][F]: Fourier coefficients (orders
    1..F) of the deviations of Gamma_1 and Gamma_2 from y = +h and y = -h."""
    F = max(1, len(g1_cos), len(g1_sin), len(g2_cos), len(g2_sin))
    out = np.zeros((2, 2, F))
    for j, (a, b) in enumerate(((g1_cos, g1_sin), (g2_cos, g2_sin))):
        out[j, 0, :len(a)] = a
        out[j, 1, :len(b)] = b
    return out


def interface_amplitude(interface) -> float:
    """Bound on |y - (+-h)| over both interfaces (sum of the coefficients' sizes)."""
    if interface is None:
        return 0.0
    return float(np.max(np.sum(np.abs(np.asarray(interface)), axis=(1, 2))))


# the interfaces of the paper's examples 1 and 2 (d = 1, h = 1):
# y = 1 + 0.1 sin(2 pi x) and y = -1 + 0.2 cos(2 pi x)
PAPER_EX12_INTERFACE = ((), (0.1,), (0.2,), ())
# and of its example 3: y = 1 + 0.05 sin(2 pi x) + 0.05 cos(2 pi x), y = -1 + 0.1 cos(2 pi x)
PAPER_EX3_INTERFACE = ((0.05,), (0.05,), (0.1,), ())


def make_problem(name, d, h, M, r_lo, r_hi, n_lo, n_hi, gap, seed, omega, phi, P,
                 n_layer=STACK, interface=None, **disc_kw) -> Problem:
    amp = interface_amplitude(interface)
    clear = None if interface is None else max(gap, 0.02) + amp
    x, y, r, n = pack_disks(M, d, h, r_lo, r_hi, n_lo, n_hi, gap, seed, clearance=clear)
    if interface is not None:
        disc_kw.setdefault("amp", amp)
    disc = derive_discretization(d, h, n_layer, omega, phi, y, P, **disc_kw)
    return Problem(d=d, h=h, n_layer=tuple(n_layer), omega=omega, phi=phi, P=P,
                   x=x, y=y, radius=r, n_incl=n, disc=disc, name=name, seed=seed,
                   interface=None if interface is None else np.asarray(interface, float))


def tiny_m4(phi=-math.pi / 5, **kw) -> Problem:
    """Plain FP64 method, M=4: d=1, middle layer y in [-0.5, 0.5], r=0.05,
    index 2.5, gap 0.02, omega=10, P=10, seed 1."""
    return make_problem("tiny_m4", 1.0, 0.5, 4, 0.05, 0.05, 2.5, 2.5, 0.02, 1,
                        10.0, phi, 10, **kw)


def m1000(phi=-math.pi / 5, **kw) -> Problem:
    """Plain FP64 method, M=1000: d=1, middle layer y in [-1, 1], radii
    U[0.004, 0.012], indices U[1.5, 3.0], gap 0.002, omega=20, P=15, seed 2."""
    return make_problem("m1000", 1.0, 1.0, 1000, 0.004, 0.012, 1.5, 3.0, 0.002, 2,
                        20.0, phi, 15, **kw)


def m1000_p20(phi=-math.pi / 5, **kw) -> Problem:
    """The M=1000 geometry (seed 2) at multipole order P=20 (41 coefficients per
    disk, generator orders up to 40)."""
    return make_problem("m1000_p20", 1.0, 1.0, 1000, 0.004, 0.012, 1.5, 3.0, 0.002, 2,
                        20.0, phi, 20, **kw)


def large_block(M=10000, R=256, seed=4, **kw):
    """Large single geometry with many incidence angles as one block of right-hand
    sides: d=4, middle layer y in [-2, 2], M disks with radii U[0.005, 0.01] and
    indices U[1.5, 3.0], gap 0.002, seed 4, omega=40, P=20; the R angles equally
    spaced in [-pi/3, pi/3].  Returns (problem at the first angle, angles)."""
    phis = np.linspace(-math.pi / 3, math.pi / 3, R)
    pb = make_problem(f"large_block_M{M}", 4.0, 2.0, M, 0.005, 0.01, 1.5, 3.0, 0.002, seed,
                      40.0, float(phis[0]), 20, **kw)
    return pb, phis


def small(M, P, omega=10.0, seed=7, phi=-math.pi / 5, d=1.0, h=0.5, **kw) -> Problem:
    """Small test geometry with m1000's size and index distributions, scaled."""
    return make_problem(f"small_M{M}_P{P}", d, h, M, 0.02, 0.04, 1.5, 3.0, 0.01, seed,
                        omega, phi, P, **kw)


def star(M, P, omega=10.0, seed=9, phi=-math.pi / 5, d=1.0, h=0.5, a2_rel=1.0 / 3.0,
         a3=3, r_lo=0.02, r_hi=0.04, n_lo=1.5, n_hi=3.0, gap=0.01, shape_nodes=64,
         **kw) -> Problem:
    """Non-circular inclusions of the paper's class (eq. par1): enclosing radii
    U[r_lo, r_hi] packed like the disks, then a1 = r / (1 + a2_rel),
    a2 = a2_rel a1, a3 lobes (the paper uses a2 / a1 = 1/3, a3 = 3), and a
    rotation U[0, 2 pi) per inclusion from a second seeded stream."""
    pb = make_problem(f"star_M{M}_P{P}", d, h, M, r_lo, r_hi, n_lo, n_hi, gap, seed, omega,
                      phi, P, **kw)
    pb.name = f"star_M{M}_P{P}"
    rng = np.random.Generator(np.random.PCG64(seed + 5_000_000))
    a1 = pb.radius / (1.0 + a2_rel)
    rot = rng.uniform(0.0, 2.0 * math.pi, size=M)
    pb.shape = np.stack([a1, a2_rel * a1, np.full(M, float(a3)), rot], axis=1)
    pb.shape_nodes = int(shape_nodes)
    return pb


def star_m1000(phi=-math.pi / 5, **kw) -> Problem:
    """The M=1000 workload's packing (seed 2, enclosing radii U[0.004, 0.012], indices
    U[1.5, 3.0], gap 0.002, omega=20, P=15) with three-lobed inclusions of eq. par1,
    a2 / a1 = 1/3, turned at random: the same enclosing circles as m1000."""
    return star(1000, 15, omega=20.0, seed=2, phi=phi, d=1.0, h=1.0, r_lo=0.004, r_hi=0.012,
                n_lo=1.5, n_hi=3.0, gap=0.002, **kw)


def empty_slab(omega=10.0, phi=-math.pi / 5, d=1.0, h=0.5, n_layer=STACK, interface=None,
               **kw) -> Problem:
    """No inclusions: the empty layered structure (flat, or with the given curved
    interfaces)."""
    e = np.zeros(0)
    if interface is not None:
        kw.setdefault("amp", interface_amplitude(interface))
    disc = derive_discretization(d, h, n_layer, omega, phi, e, 10, **kw)
    return Problem(d=d, h=h, n_layer=tuple(n_layer), omega=omega, phi=phi, P=10,
                   x=e, y=e.copy(), radius=e.copy(), n_incl=e.copy(), disc=disc,
                   name="empty" if interface is None else "empty_curved",
                   interface=None if interface is None else np.asarray(interface, float))


def curved(M, P, omega=10.0, seed=7, phi=-math.pi / 5, d=1.0, h=0.5,
           interface=((), (0.05,), (0.04,), (0.02,)), **kw) -> Problem:
    """small()'s inclusions between curved interfaces (default Gamma_1:
    y = h + 0.05 sin(2 pi x), Gamma_2: y = -h + 0.04 cos(2 pi x) + 0.02 sin(2 pi x));
    the packing keeps every disk at least 0.02 + the interfaces' amplitude from
    y = +-h."""
    pb = make_problem(f"curved_M{M}_P{P}", d, h, M, 0.02, 0.04, 1.5, 3.0, 0.01, seed,
                      omega, phi, P, interface=interface_profile(*interface), **kw)
    return pb


def lossy(M, P, omega=10.0, seed=7, phi=-math.pi / 5, loss=(0.05, 0.5), **kw) -> Problem:
    """small()'s geometry with absorbing inclusions: the imaginary parts of the
    indices U[loss] from a second seeded stream (seed + 6000000)."""
    pb = small(M, P, omega=omega, seed=seed, phi=phi, **kw)
    pb.name = f"lossy_M{M}_P{P}"
    rng = np.random.Generator(np.random.PCG64(seed + 6_000_000))
    pb.n_incl_im = rng.uniform(loss[0], loss[1], size=M)
    return pb


def lossy_substrate(M, P, omega=10.0, seed=7, phi=-math.pi / 5, n3_im=0.05,
                    curved_iface=False, **kw) -> Problem:
    """small()'s geometry (or curved()'s with curved_iface) over an absorbing
    substrate: the bottom layer's index n_3 + i n3_im."""
    if curved_iface:
        pb = curved(M, P, omega=omega, seed=seed, phi=phi, **kw)
    else:
        pb = small(M, P, omega=omega, seed=seed, phi=phi, **kw)
    pb.name = f"substrate_M{M}_P{P}" + ("_curved" if curved_iface else "")
    pb.n3_im = float(n3_im)
    return pb


def curved_m1000(phi=-math.pi / 5, **kw) -> Problem:
    """The M=1000 workload's rules (d=1, h=1, radii U[0.004, 0.012], indices
    U[1.5, 3.0], gap 0.002, omega=20, P=15, seed 2) between the interfaces of the
    paper's examples 1 and 2, y = 1 + 0.1 sin(2 pi x) and y = -1 + 0.2 cos(2 pi x)."""
    return make_problem("curved_m1000", 1.0, 1.0, 1000, 0.004, 0.012, 1.5, 3.0, 0.002, 2,
                        20.0, phi, 15, interface=interface_profile(*PAPER_EX12_INTERFACE),
                        **kw)


# ----------------------------------------------------------------------------
# learned warm start: geometry sets, initial weights, synthetic targets
# ----------------------------------------------------------------------------

WARM_OMEGAS = (10.0, 20.0, 30.0, 40.0)
WARM_PHIS = (-math.pi / 3, -math.pi / 9, math.pi / 9, math.pi / 3)


def warm_problem(i: int, held_out: bool = False, M_range=(200, 2000), P: int = 20,
                 omegas=WARM_OMEGAS, phis=WARM_PHIS) -> Problem:
    """Geometry i of the warm-start training set (seed 50000+i) or of the held-out
    set (seed 90000+i): the M=1000 workload's rules (d=1, middle layer y in [-1, 1],
    radii U[0.004, 0.012], indices U[1.5, 3.0], gap 0.002) with M a seeded uniform
    integer in M_range, P = 20, and (omega, phi) taken in turn from a grid over
    omega in [10, 40] and phi in [-pi/3, pi/3] (omega fastest).  All problems with the
    same (omega, phi) get the same discretization (interface nodes from the closest
    position the packing allows), so they share one factorization of the layers."""
    seed = (90000 if held_out else 50000) + i
    rng = np.random.Generator(np.random.PCG64(seed + 7_000_000))
    M = int(rng.integers(M_range[0], M_range[1] + 1))
    omega = float(omegas[i % len(omegas)])
    phi = float(phis[(i // len(omegas)) % len(phis)])
    d, h, r_lo, gap = 1.0, 1.0, 0.004, 0.002
    x, y, r, n = pack_disks(M, d, h, r_lo, 0.012, 1.5, 3.0, gap, seed)
    closest = h - (max(gap, 0.02) + r_lo)
    disc = derive_discretization(d, h, STACK, omega, phi, np.array([closest]), P)
    return Problem(d=d, h=h, n_layer=STACK, omega=omega, phi=phi, P=P, x=x, y=y, radius=r,
                   n_incl=n, disc=disc, name=f"warm{'H' if held_out else 'T'}{i}_M{M}",
                   seed=seed)


BATCH_OMEGAS = (10.0, 20.0, 40.0)
BATCH_PHIS = tuple(-math.pi / 3 + a * (2 * math.pi / 3) / 15 for a in range(16))
BATCH_PS = (10, 15, 20)


def batch_problem(i: int, cells=None) -> Problem:
    """Instance i of the batched mixed-precision workload (seed 3000+i): the M=1000
    workload's rules (d=1, middle layer y in [-1, 1], radii U[0.004, 0.012], indices
    U[1.5, 3.0], gap 0.002) with M log-uniform in [200, 4000], at the (omega, phi) cell
    i mod len(cells) of the grid omega in {10, 20, 40} x 16 angles equally spaced in
    [-pi/3, pi/3] (cells: list of (omega index, phi index); default the whole grid with
    omega fastest, so instance i has omega index i mod 3 and angle index (i div 3) mod
    16).  The multipole order goes with the frequency as in the single-problem
    workloads: P = 10, 15, 20 at omega = 10, 20, 40.  Problems of one cell share their
    discretization, hence one factorization of the layered structure."""
    if cells is None:
        cells = [(w, a) for a in range(len(BATCH_PHIS)) for w in range(len(BATCH_OMEGAS))]
    wi, ai = cells[i % len(cells)]
    omega, phi = BATCH_OMEGAS[wi], BATCH_PHIS[ai]
    P = int(BATCH_PS[wi])
    seed = 3000 + i
    rng = np.random.Generator(np.random.PCG64(seed + 7_000_000))
    M = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
    d, h, r_lo, gap = 1.0, 1.0, 0.004, 0.002
    x, y, r, n = pack_disks(M, d, h, r_lo, 0.012, 1.5, 3.0, gap, seed)
    closest = h - (max(gap, 0.02) + r_lo)
    disc = derive_discretization(d, h, STACK, omega, phi, np.array([closest]), P)
    return Problem(d=d, h=h, n_layer=STACK, omega=omega, phi=phi, P=P, x=x, y=y, radius=r,
                   n_incl=n, disc=disc, name=f"batch{i}_M{M}_P{P}", seed=seed)


def nn_shapes(H: int, L: int, p_out: int, F: int = 32, E: int = 8):
    """Shapes of the warm-start network's weights, in the order of its flat
    parameter vector (matrices row-major [rows][cols])."""
    O = 2 * (2 * p_out + 1)
    s = [(H, F), (H,)]
    for _ in range(L):
        s += [(H, H), (H, H), (H, E), (H,), (H, 2 * H), (H,)]
    s += [(O, H), (O,)]
    return s


def nn_init(H: int, L: int, p_out: int, seed: int = 0, out_scale: float = 0.1):
    """Seeded initial weights (float32): uniform in +-sqrt(6 / fan_in) for
    matrices (scaled by out_scale for the output layer), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = nn_shapes(H, L, p_out)
    parts = []
    for i, s in enumerate(shapes):
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            a = math.sqrt(6.0 / s[1]) * (out_scale if i == len(shapes) - 2 else 1.0)
            parts.append(rng.uniform(-a, a, size=s))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def nn_synthetic_target(M: int, p_out: int, seed: int = 0):
    """Seeded target t, positive weights w ([M][2(2 p_out + 1)] float32) and a
    normaliser, for checks of the loss and its gradient."""
    rng = np.random.Generator(np.random.PCG64(seed))
    O = 2 * (2 * p_out + 1)
    t = rng.standard_normal((M, O)).astype(np.float32)
    w = rng.uniform(0.1, 1.0, size=(M, O)).astype(np.float32)
    w[:, 1::2] = w[:, 0::2]
    return t, w, float(M * O)
