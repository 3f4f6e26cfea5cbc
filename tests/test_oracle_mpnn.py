"""Pins of the warm-start network reference (oracle/mpnn.py), CPU only."""
import math

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from oracle import mpnn


def test_bf16_rounding_by_definition():
    one = 1.0
    # bfloat16 has 7 fraction bits: neighbours of 1 are 1 + k 2^-7
    assert mpnn.bf16_round(one) == 1.0
    assert mpnn.bf16_round(1 + 2.0 ** -8) == 1.0                 # tie -> even (k = 0)
    assert mpnn.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6   # tie -> even (k = 2)
    assert mpnn.bf16_round(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert mpnn.bf16_round(-(1 + 2.0 ** -8 + 2.0 ** -20)) == -(1 + 2.0 ** -7)
    assert mpnn.bf16_round(3.0) == 3.0
    a = np.random.default_rng(1).standard_normal(1000)
    r = mpnn.bf16_round(a)
    assert np.array_equal(mpnn.bf16_round(r), r)                # idempotent
    assert np.max(np.abs(r - a) / np.abs(a)) <= 2.0 ** -8        # half an ulp


def test_param_layout_matches_inputs():
    H, L, p = 16, 2, 3
    shapes = [s for _, s in mpnn.param_layout(H, L, p)]
    assert shapes == [tuple(s) for s in inputs.nn_shapes(H, L, p)]
    assert mpnn.n_params(H, L, p) == inputs.nn_init(H, L, p).size


def test_knn_brute_force_with_wrap():
    rng = np.random.default_rng(3)
    M, K, d = 30, 5, 1.0
    x = rng.uniform(-0.5, 0.5, M)
    y = rng.uniform(-0.3, 0.3, M)
    x[0], y[0] = 0.495, 0.0
    x[1], y[1] = -0.495, 0.001           # 0.01 away through the wall
    nbr = mpnn.knn(x, y, d, K)
    for j in range(M):
        dist = []
        for m in range(M):
            if m == j:
                continue
            dxs = [x[j] - x[m] + s * d for s in (-1, 0, 1)]
            dx = min(dxs, key=abs)
            dist.append((math.hypot(dx, y[j] - y[m]), m))
        dist.sort()
        assert [m for _, m in dist[:K]] == list(nbr[j])
    assert nbr[0, 0] == 1 and nbr[1, 0] == 0
    # fewer than K others: padded with -1
    nb2 = mpnn.knn(x[:3], y[:3], d, K)
    assert (nb2[:, 2:] == -1).all() and (nb2[:, :2] >= 0).all()


def test_edge_features_table_values():
    """z = 1 along +x: Hankel values from the printed tables of J and Y at 1."""
    k2 = 10.0

    class Pb:
        pass
    pb = Pb()
    pb.d = 1.0
    pb.x = np.array([0.05, -0.05])
    pb.y = np.array([0.0, 0.0])
    e = mpnn.edge_features(pb, np.array([[1], [0]]), k2)
    J0, Y0, J1, Y1 = 0.7651976866, 0.0882569642, 0.4400505857, -0.7812128213
    np.testing.assert_allclose(e[0, 0], [1.0, 0.0, 1.0, 1.0, J0, Y0, J1, Y1], atol=1e-9)
    # the reverse edge points along -x: e^{i phi} = -1
    np.testing.assert_allclose(e[1, 0], [-1.0, 0.0, 1.0, 1.0, J0, Y0, -J1, -Y1], atol=1e-9)


def _tiny_net(M=9, K=4, H=8, L=2, p=2, seed=5):
    rng = np.random.default_rng(seed)
    feat = rng.standard_normal((M, mpnn.F_NODE))
    x = rng.uniform(-0.5, 0.5, M)
    y = rng.uniform(-0.4, 0.4, M)
    nbr = mpnn.knn(x, y, 1.0, K)
    edge = rng.standard_normal((M, K, mpnn.E_EDGE))
    theta = inputs.nn_init(H, L, p, seed=seed, out_scale=1.0).astype(np.float64)
    # biases nonzero so every term of the gradient is exercised
    theta += 0.05 * rng.standard_normal(theta.size)
    t, w, wn = inputs.nn_synthetic_target(M, p, seed)
    return feat, nbr, edge, theta, t.astype(float), w.astype(float), wn, H, L, p


def test_gradient_central_differences():
    feat, nbr, edge, theta, t, w, wn, H, L, p = _tiny_net()
    out, cache = mpnn.forward(theta, feat, nbr, edge, H, L, p)
    g = mpnn.backward(theta, feat, nbr, edge, H, L, p, cache, out, t, w, wn)
    rng = np.random.default_rng(0)
    idx = rng.choice(theta.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp = mpnn.loss(mpnn.forward(tp, feat, nbr, edge, H, L, p)[0], t, w, wn)
        lm = mpnn.loss(mpnn.forward(tm, feat, nbr, edge, H, L, p)[0], t, w, wn)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_node_order_equivariance():
    feat, nbr, edge, theta, t, w, wn, H, L, p = _tiny_net()
    M = feat.shape[0]
    perm = np.random.default_rng(2).permutation(M)
    inv = np.argsort(perm)
    nbr_p = np.where(nbr[perm] >= 0, inv[np.where(nbr[perm] >= 0, nbr[perm], 0)], -1)
    o1, _ = mpnn.forward(theta, feat, nbr, edge, H, L, p)
    o2, _ = mpnn.forward(theta, feat[perm], nbr_p, edge[perm], H, L, p)
    np.testing.assert_allclose(o2, o1[perm], rtol=1e-12, atol=1e-12)


@pytest.fixture(scope="module")
def small_solved():
    from oracle.solver import Reduced
    pb = inputs.small(20, 6, seed=61)
    red = Reduced(pb)
    beta = red.solve_lu()
    return pb, red, beta


def test_exact_correction_reproduces_solution(small_solved):
    """beta* = s (alpha0 + (T beta* - B_phys A^+ C beta*)): with the exact
    correction on every order the warm start is the solution; with none it is b."""
    pb, red, beta = small_solved
    a0 = mpnn.incident(red)
    t, w, wn = mpnn.targets(red, beta, a0, pb.P)
    x0 = mpnn.warm_start(red, a0, t, pb.P)
    assert np.linalg.norm(x0 - beta) / np.linalg.norm(beta) < 1e-10
    xb = mpnn.warm_start(red, a0, np.zeros_like(t), pb.P)
    assert np.linalg.norm(xb - red.rhs()) <= 1e-14 * np.linalg.norm(xb)
    # the loss of the exact correction is 0 and of no correction is the
    # normalised error of the single-scattering guess on those orders
    assert mpnn.loss(t, t, w, wn) == 0.0
    assert 0 < mpnn.loss(np.zeros_like(t), t, w, wn) < 1


def test_node_features_shape_and_values(small_solved):
    pb, red, beta = small_solved
    a0 = mpnn.incident(red)
    f = mpnn.node_features(red, a0)
    P = pb.P
    nb = 2 * P + 1
    assert f.shape == (pb.M, mpnn.F_NODE)
    np.testing.assert_allclose(f[:, 0], red.G.k2 * pb.radius)
    np.testing.assert_allclose(f[:, 11 + 6] + 1j * f[:, 12 + 6], a0.reshape(-1, nb)[:, P])
    assert np.all(f[:, 25:] == 0)
