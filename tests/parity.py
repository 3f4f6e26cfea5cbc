"""Per-order comparison of coefficient vectors in the normalised basis.

Multipole coefficients of small disks span dozens of decades across the orders
n = -P..P (an outgoing coefficient of order n scales like 1/|H_n(k2 r)|), so one
2-norm over a whole vector only checks its largest orders.  Every parity test
therefore compares order by order in the basis normalised by
D_m[n] = |H_|n|(k2 r_m)| (the size of the multipole on its own disk boundary):
for each order n,

    err_n   = max_j |D (y - y_ref)|_{j,n}
    scale_n = max_j |D y_ref|_{j,n}

and requires err_n <= rtol * scale_n + atol * max_n scale_n.  Apply outputs
(deterministic sums) use atol = 0: every order is held to rtol of its own size.
Iterative solutions use atol = 1e-10: a solve to a normalised residual of 1e-12
bounds the error by about cond(D K D^-1) * 1e-12 of the whole vector, which says
nothing about an order 1e-13 below the largest one.  Vectors computed through the
pseudo-inverse alone (the right-hand side S B_phys A^+ f) use atol = 1e-12: the
singular-value cut at 1e-10 fixes A^+ f only to about that level, and its error
reaches high orders that are 1e-14 of the largest.

D is computed here from SciPy's Hankel function (independent of the library).
"""
import numpy as np
import scipy.special as sp


def dscale(pb):
    """D = |H_|n|(k2 r_m)| as a flat [M (2P+1)] vector."""
    P = int(pb.P)
    k2 = pb.omega * pb.n_layer[1]
    n = np.abs(np.arange(-P, P + 1))
    r = np.asarray(pb.radius, float)
    return np.abs(sp.hankel1(n[None, :], k2 * r[:, None])).reshape(-1)


def probe(pb, seed):
    """x = D^-1 u with u standard complex normal in every order (flat, complex)."""
    D = dscale(pb)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(D.size) + 1j * rng.standard_normal(D.size)
    return u / D


def order_errors(y, y_ref, D, P):
    nb = 2 * P + 1
    e = np.abs(D * (np.asarray(y) - np.asarray(y_ref))).reshape(-1, nb).max(axis=0)
    s = np.abs(D * np.asarray(y_ref)).reshape(-1, nb).max(axis=0)
    return e, s


def check_orders(y, y_ref, D, P, rtol, atol=0.0, tag=""):
    """Assert the per-order bound; return the worst per-order relative error."""
    e, s = order_errors(y, y_ref, D, P)
    bound = rtol * s + atol * s.max()
    ratio = e / np.maximum(s, 1e-300)
    worst = float(ratio.max())
    bad = np.nonzero(e > bound)[0]
    print(f"[orders] {tag} P={P}: worst per-order rel err {worst:.2e} "
          f"(order {int(np.argmax(ratio)) - P}); scales {s.min():.1e}..{s.max():.1e}",
          flush=True)
    assert bad.size == 0, (f"{tag}: orders {[int(b) - P for b in bad]} exceed the bound: "
                           f"err {e[bad]} scale {s[bad]}")
    return worst


def check_amplitudes(c, c_ref, rtol, atol=1e-12, tag=""):
    """Bragg amplitudes (propagating orders only): |c - c_ref|_n <= rtol |c_ref,n|
    + atol max |c_ref| for every order n."""
    c = np.asarray(c)
    c_ref = np.asarray(c_ref)
    e = np.abs(c - c_ref)
    s = np.abs(c_ref)
    bound = rtol * s + atol * s.max()
    worst = float((e / np.maximum(s, 1e-300)).max()) if s.size else 0.0
    print(f"[amplitudes] {tag}: {s.size} propagating, worst rel err {worst:.2e}, "
          f"|c| {s.min() if s.size else 0:.1e}..{s.max() if s.size else 0:.1e}", flush=True)
    assert np.all(e <= bound), (tag, e, s)
    return worst
