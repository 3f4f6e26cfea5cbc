"""Reference of the learned warm start: features, message-passing network, loss
and gradients, in FP64 NumPy (oracle).

Test infrastructure only (see oracle/__init__.py).

The network predicts, for every inclusion j, a correction to the incoming-field
coefficients of the empty layered structure, alpha0_j = (B_phys A^+ f)_j (the field
the layers alone send to inclusion j, sec. 5), so that the GMRES initial guess is

    beta0_j[n] = s_j[n] (alpha0_j[n] + out_j[n]),   |n| <= p_out,

and s_j[n] alpha0_j[n] for the other orders (single scattering).  The exact
correction is the multiple-scattering part of the incoming field,
alpha*_j - alpha0_j = (T beta* - B_phys A^+ C beta*)_j, since beta* = S alpha*.

Graph: each inclusion's K nearest other inclusions under the minimum-image
distance in x (period d), ties broken by index; missing neighbours (M - 1 < K)
are marked -1.

Network (width H, L layers, F = 32 node inputs, E = 8 edge inputs,
O = 2 (2 p_out + 1) outputs), all weights in one flat vector:

    h0_j   = relu(W_in f_j + b_in)
    layer: P_j = A h_j, Q_j = B h_j
           msg_jk = relu(P_j + Q_{nbr(j,k)} + C e_jk + c)
           agg_j  = mean over the valid k of msg_jk (0 if none)
           h_j   <- h_j + relu(U [h_j; agg_j] + u)
    out_j  = W_out h_j + b_out

Flat layout (row-major matrices [rows][cols]): W_in [H][F], b_in [H]; per layer
A [H][H], B [H][H], C [H][E], c [H], U [H][2H], u [H]; then W_out [O][H],
b_out [O].  out_j holds (Re, Im) pairs for n = -p_out .. p_out.

Loss of one geometry: sum_j,n w_jn |out_jn - t_jn|^2 / wnorm with w_jn =
(D_jn |s_jn|)^2 (D the normalisation of the reduced system), t the exact
correction and wnorm = sum_j,n w_jn |alpha*_jn|^2: the squared relative error of
the normalised initial guess restricted to the predicted orders.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

F_NODE = 32
E_EDGE = 8


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), via float32; returns float64.

    bfloat16 keeps the upper 16 bits of the IEEE float32 pattern; rounding adds
    0x7FFF plus the lowest kept bit before truncating."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def param_layout(H, L, p_out):
    """[(name, shape)] in flat order."""
    O = 2 * (2 * p_out + 1)
    out = [("W_in", (H, F_NODE)), ("b_in", (H,))]
    for l in range(L):
        out += [(f"A{l}", (H, H)), (f"B{l}", (H, H)), (f"C{l}", (H, E_EDGE)), (f"c{l}", (H,)),
                (f"U{l}", (H, 2 * H)), (f"u{l}", (H,))]
    out += [("W_out", (O, H)), ("b_out", (O,))]
    return out


def n_params(H, L, p_out):
    return int(sum(np.prod(s) for _, s in param_layout(H, L, p_out)))


def unpack(theta, H, L, p_out):
    d, o = {}, 0
    for name, shape in param_layout(H, L, p_out):
        n = int(np.prod(shape))
        d[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return d


def pack(d, H, L, p_out):
    return np.concatenate([np.asarray(d[name]).reshape(-1) for name, _ in
                           param_layout(H, L, p_out)])


# ----------------------------------------------------------------------------
# graph and features
# ----------------------------------------------------------------------------

def min_image_dx(xj, xm, d):
    dx = xj - xm
    dx = np.where(dx > d / 2, dx - d, dx)
    dx = np.where(dx < -d / 2, dx + d, dx)
    return dx


def knn(x, y, d, K):
    """Neighbour indices [M][K] (-1 where fewer than K others exist)."""
    M = len(x)
    nbr = -np.ones((M, K), dtype=np.int64)
    for j in range(M):
        dx = min_image_dx(x[j], x, d)
        dy = y[j] - y
        r2 = dx * dx + dy * dy
        idx = np.array([m for m in range(M) if m != j], dtype=np.int64)
        order = np.lexsort((idx, r2[idx]))
        cnt = min(K, M - 1)
        nbr[j, :cnt] = idx[order[:cnt]]
    return nbr


def incident(red):
    """alpha0 = B_phys A^+ f: incoming coefficients from the layers alone."""
    return red.B @ red.pinv.apply(red.f)


def node_features(red, alpha0):
    G, pb = red.G, red.G.pb
    M, P = G.M, G.P
    nb = 2 * P + 1
    s = red.s.reshape(M, nb)
    D = red.D.reshape(M, nb)
    a0 = alpha0.reshape(M, nb)
    f = np.zeros((M, F_NODE))
    f[:, 0] = G.k2 * G.rad
    f[:, 1] = pb.n_incl / pb.n_layer[1] - 1.0
    f[:, 2] = pb.y / pb.h
    f[:, 3] = np.sin(pb.phi)
    f[:, 4] = pb.omega / 40.0
    for n in range(3):
        if n <= P:
            v = D[:, P + n] * s[:, P + n]
            f[:, 5 + 2 * n] = v.real
            f[:, 6 + 2 * n] = v.imag
    for n in range(-3, 4):
        if abs(n) <= P:
            f[:, 11 + 2 * (n + 3)] = a0[:, P + n].real
            f[:, 12 + 2 * (n + 3)] = a0[:, P + n].imag
    return f


def edge_features(pb, nbr, k2):
    M, K = nbr.shape
    e = np.zeros((M, K, E_EDGE))
    for j in range(M):
        for k in range(K):
            m = nbr[j, k]
            if m < 0:
                continue
            dx = float(min_image_dx(pb.x[j], pb.x[m], pb.d))
            dy = pb.y[j] - pb.y[m]
            rho = np.hypot(dx, dy)
            z = k2 * rho
            eph = (dx + 1j * dy) / rho
            h0 = sp.hankel1(0, z)
            h1 = sp.hankel1(1, z) * eph
            e[j, k] = [k2 * dx, k2 * dy, z, 1.0 / z, h0.real, h0.imag, h1.real, h1.imag]
    return e


def targets(red, beta, alpha0, p_out):
    """Exact correction t, weights w and wnorm for a solved geometry."""
    G = red.G
    M, P = G.M, G.P
    nb = 2 * P + 1
    corr = (red.T_apply(beta) - red.lowrank_apply(beta)).reshape(M, nb)
    a0 = alpha0.reshape(M, nb)
    s = red.s.reshape(M, nb)
    D = red.D.reshape(M, nb)
    O = 2 * (2 * p_out + 1)
    t = np.zeros((M, O))
    w = np.zeros((M, O))
    wnorm = 0.0
    for n in range(-p_out, p_out + 1):
        if abs(n) > P:
            continue
        i = 2 * (n + p_out)
        t[:, i] = corr[:, P + n].real
        t[:, i + 1] = corr[:, P + n].imag
        ww = (D[:, P + n] * np.abs(s[:, P + n])) ** 2
        w[:, i] = ww
        w[:, i + 1] = ww
        wnorm += float(np.sum(ww * np.abs(a0[:, P + n] + corr[:, P + n]) ** 2))
    return t, w, wnorm


def warm_start(red, alpha0, out, p_out):
    """beta0 = s (alpha0 + out) on the predicted orders, s alpha0 elsewhere."""
    G = red.G
    M, P = G.M, G.P
    nb = 2 * P + 1
    a = alpha0.reshape(M, nb).copy()
    for n in range(-p_out, p_out + 1):
        if abs(n) <= P:
            i = 2 * (n + p_out)
            a[:, P + n] += out[:, i] + 1j * out[:, i + 1]
    return red.s * a.reshape(-1)


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------

def _relu(v):
    return np.maximum(v, 0.0)


def forward(theta, feat, nbr, edge, H, L, p_out):
    """Outputs [M][O] and the intermediate values the backward pass needs."""
    p = unpack(theta, H, L, p_out)
    valid = nbr >= 0
    cnt = valid.sum(axis=1)
    inv = np.where(cnt > 0, 1.0 / np.maximum(cnt, 1), 0.0)
    nbr_c = np.where(valid, nbr, 0)
    pre0 = feat @ p["W_in"].T + p["b_in"]
    h = _relu(pre0)
    cache = {"pre0": pre0, "h": [h], "layers": []}
    for l in range(L):
        Pj = h @ p[f"A{l}"].T
        Qj = h @ p[f"B{l}"].T
        pre = Pj[:, None, :] + Qj[nbr_c] + edge @ p[f"C{l}"].T + p[f"c{l}"]
        msg = _relu(pre) * valid[:, :, None]
        agg = msg.sum(axis=1) * inv[:, None]
        z = np.concatenate([h, agg], axis=1)
        upre = z @ p[f"U{l}"].T + p[f"u{l}"]
        h = h + _relu(upre)
        cache["layers"].append({"pre": pre, "agg": agg, "z": z, "upre": upre})
        cache["h"].append(h)
    out = h @ p["W_out"].T + p["b_out"]
    return out, cache


def loss(out, t, w, wnorm):
    return float(np.sum(w * (out - t) ** 2) / wnorm)


def backward(theta, feat, nbr, edge, H, L, p_out, cache, out, t, w, wnorm):
    """Gradient of loss() with respect to theta (same flat layout)."""
    p = unpack(theta, H, L, p_out)
    g = {k: np.zeros_like(v) for k, v in p.items()}
    valid = nbr >= 0
    cnt = valid.sum(axis=1)
    inv = np.where(cnt > 0, 1.0 / np.maximum(cnt, 1), 0.0)
    nbr_c = np.where(valid, nbr, 0)
    dout = 2.0 * w * (out - t) / wnorm
    hL = cache["h"][L]
    g["W_out"] = dout.T @ hL
    g["b_out"] = dout.sum(axis=0)
    dh = dout @ p["W_out"]
    for l in reversed(range(L)):
        c = cache["layers"][l]
        h = cache["h"][l]
        dupre = dh * (c["upre"] > 0)
        g[f"U{l}"] = dupre.T @ c["z"]
        g[f"u{l}"] = dupre.sum(axis=0)
        dz = dupre @ p[f"U{l}"]
        dh = dh + dz[:, :H]
        dagg = dz[:, H:]
        dmsg = (dagg * inv[:, None])[:, None, :] * (c["pre"] > 0) * valid[:, :, None]
        dP = dmsg.sum(axis=1)
        dQ = np.zeros_like(dP)
        np.add.at(dQ, nbr_c[valid], dmsg[valid])
        g[f"C{l}"] = np.einsum("jkc,jke->ce", dmsg, edge)
        g[f"c{l}"] = dmsg.sum(axis=(0, 1))
        g[f"A{l}"] = dP.T @ h
        g[f"B{l}"] = dQ.T @ h
        dh = dh + dP @ p[f"A{l}"] + dQ @ p[f"B{l}"]
    dpre0 = dh * (cache["pre0"] > 0)
    g["W_in"] = dpre0.T @ feat
    g["b_in"] = dpre0.sum(axis=0)
    return pack(g, H, L, p_out)
