"""Learned warm start on the GPU (grt_nn_*) against the FP64 reference of
oracle/mpnn.py.

Bars: neighbour lists exact; node and edge inputs, which the library stores in
FP32, within FP32 rounding of the oracle's FP64 values; outputs, loss and
gradients of the network on the same bfloat16-rounded weights within 1e-4
relative (FP32 accumulation against FP64); warm-started solves reach the cold
solution to 1e-9.
"""
import math
import sys

import numpy as np
import pytest

from paper_1412_7466_amd import inputs

pytestmark = pytest.mark.gpu

H, L, K, P_OUT = 128, 3, 16, 3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def _ctx(pb):
    from paper_1412_7466_amd.grating import Context
    say(f"[gpu] nn case {pb.name} M={pb.M} P={pb.P}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return ctx


@pytest.fixture(scope="module")
def cases(torch_cuda):
    from oracle.solver import Reduced
    out = []
    for pb in (inputs.small(20, 6, seed=61), inputs.small(12, 4, seed=21)):
        red = Reduced(pb)
        ctx = _ctx(pb)
        beta, _ = ctx.solve(tol=1e-12, restart=150)
        out.append((pb, red, ctx, beta, red.solve_lu()))
    return out


def test_incident_matches_oracle(cases):
    from oracle import mpnn
    for pb, red, ctx, beta, beta_o in cases:
        a = ctx.incident().cpu().numpy()
        assert rel(a, mpnn.incident(red)) < 1e-9


def test_graph_inputs_and_target_match_oracle(cases):
    from oracle import mpnn
    from paper_1412_7466_amd.grating import Network
    net = Network(H, L, K, P_OUT)
    for pb, red, ctx, beta, beta_o in cases:
        i = net.add_sample(ctx, beta)
        s = net.sample(i)
        a0 = mpnn.incident(red)
        nbr = mpnn.knn(pb.x, pb.y, pb.d, K)
        assert np.array_equal(s["nbr"], nbr)
        feat = mpnn.node_features(red, a0)
        np.testing.assert_allclose(s["feat"], feat, rtol=1e-6, atol=1e-6)
        edge = mpnn.edge_features(pb, nbr, red.G.k2)
        np.testing.assert_allclose(s["edge"], edge, rtol=1e-6, atol=1e-6)
        t, w, wn = mpnn.targets(red, beta_o, a0, P_OUT)
        np.testing.assert_allclose(s["weight"], w, rtol=1e-6, atol=1e-30)
        assert rel(s["target"], t) < 1e-6
        assert abs(s["wnorm"] / wn - 1) < 1e-8
    net.close()


def test_forward_and_gradient_match_oracle(cases):
    """Same weights (rounded to bfloat16), same seeded target: outputs, loss and the
    gradient of every weight tensor against the FP64 reference."""
    from oracle import mpnn
    from paper_1412_7466_amd.grating import Network
    net = Network(H, L, K, P_OUT)
    theta = inputs.nn_init(H, L, P_OUT, seed=11, out_scale=1.0)
    rng = np.random.default_rng(12)
    theta = (theta + 0.05 * rng.standard_normal(theta.size)).astype(np.float32)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    th = mpnn.bf16_round(theta)
    for pb, red, ctx, beta, beta_o in cases:
        i = net.add_sample(ctx)
        t, w, wn = inputs.nn_synthetic_target(pb.M, P_OUT, seed=pb.M)
        net.set_target(i, t, w, wn)
        loss, g, out = net.loss_grad(i)
        # the oracle's own inputs, stored as FP32 like the library's
        a0 = mpnn.incident(red)
        nbr = mpnn.knn(pb.x, pb.y, pb.d, K)
        feat = mpnn.node_features(red, a0).astype(np.float32).astype(np.float64)
        edge = mpnn.edge_features(pb, nbr, red.G.k2).astype(np.float32).astype(np.float64)
        oo, cache = mpnn.forward(th, feat, nbr, edge, H, L, P_OUT)
        lo = mpnn.loss(oo, t.astype(float), w.astype(float), wn)
        go = mpnn.backward(th, feat, nbr, edge, H, L, P_OUT, cache, oo, t.astype(float),
                           w.astype(float), wn)
        say(f"[gpu] nn M={pb.M}: out {rel(out, oo):.2e} loss {abs(loss / lo - 1):.2e} "
            f"grad {rel(g, go):.2e}")
        assert rel(out, oo) < 1e-4
        assert abs(loss / lo - 1) < 1e-4
        assert rel(g, go) < 1e-4
        off = 0
        for name, shape in mpnn.param_layout(H, L, P_OUT):
            n = int(np.prod(shape))
            e = rel(g[off:off + n], go[off:off + n])
            assert e < 1e-3, (name, e)
            off += n
        # the initial guess beta0 = s (alpha0 + out) from the same weights
        x0 = net.predict(ctx).cpu().numpy()
        x0o = mpnn.warm_start(red, a0, oo, P_OUT)
        assert rel(x0, x0o) < 1e-4
    net.close()


def test_training_reduces_loss_and_warm_start_is_exact(cases, torch_cuda):
    from oracle import mpnn
    from paper_1412_7466_amd.grating import Network
    net = Network(H, L, K, P_OUT)
    net.set_params(inputs.nn_init(H, L, P_OUT, seed=3))
    ids = [net.add_sample(ctx, beta) for pb, red, ctx, beta, beta_o in cases]
    l0 = np.mean([net.loss_grad(i)[0] for i in ids])
    l1 = net.train(ids, epochs=60, lr=1e-3, seed=1)
    l2 = np.mean([net.loss_grad(i)[0] for i in ids])
    say(f"[gpu] nn loss {l0:.3e} -> {l2:.3e} (last epoch mean {l1:.3e})")
    assert l2 < 0.5 * l0
    for pb, red, ctx, beta, beta_o in cases:
        x0 = net.predict(ctx)
        bw, sw = ctx.solve(tol=1e-12, restart=150, x0=x0)
        assert sw.x0_rejected == 0
        assert rel(bw.cpu().numpy(), beta_o) < 1e-9
    net.close()


def test_bad_guess_is_dropped(cases, torch_cuda):
    pb, red, ctx, beta, beta_o = cases[0]
    rng = np.random.default_rng(0)
    junk = 1e3 * (rng.standard_normal(red.G.n_beta) + 1j * rng.standard_normal(red.G.n_beta))
    x0 = torch_cuda.tensor(junk, dtype=torch_cuda.complex128, device="cuda:0")
    b, st = ctx.solve(tol=1e-12, restart=150, x0=x0)
    assert st.x0_rejected == 1
    assert rel(b.cpu().numpy(), beta_o) < 1e-9
