"""TE polarisation on the GPU (u = H_z: u and (1/eps) du/dn continuous; the paper
treats TM only) against the CPU oracle's TE (pinned in tests/test_oracle_te.py).

The library assembles A with the TE factors, computes the TE Mie coefficients and
folds the flux-row and potential factors of C and B_phys into its pseudo-inverse
factors, so the apply kernels run unchanged.  Bars as for TM (tests/test_gpu_parity.py):
equilibrated A to 1e-12, the Mie diagonal per order 1e-11, T 1e-12, K, the right-hand
side, solutions and Bragg amplitudes 1e-9, flux 1e-10.
"""
import math
import sys

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from parity import check_amplitudes, check_orders, dscale, probe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def _te(pb):
    pb.polarization = "TE"
    return pb


def _ctx(pb):
    from paper_1412_7466_amd.grating import Context
    say(f"[gpu] TE case {pb.name} M={pb.M} P={pb.P} phi={pb.phi:.4f}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return ctx


def _np(t):
    return t.detach().cpu().numpy()


def _bragg(og, oo, tag):
    vg = np.concatenate([og["c"][oo["prop1"]], og["d"][oo["prop3"]]])
    vo = np.concatenate([oo["c"][oo["prop1"]], oo["d"][oo["prop3"]]])
    check_amplitudes(vg, vo, 1e-9, tag=tag)


@pytest.mark.parametrize("phi", [-math.pi / 5, 0.3])
def test_te_empty_slab(torch_cuda, phi):
    from oracle.solver import Reduced
    pb = _te(inputs.empty_slab(phi=phi))
    red = Reduced(pb)
    ctx = _ctx(pb)
    og = ctx.bragg()
    oo = red.bragg(np.zeros(0))
    i0 = list(oo["orders"]).index(0)
    assert abs(og["c"][i0] - oo["c"][i0]) < 1e-12
    assert abs(og["d"][i0] - oo["d"][i0]) < 1e-12
    assert og["flux_err"] < 1e-12
    ctx.close()


@pytest.mark.parametrize("case", ["tiny", "small"])
def test_te_pieces_and_solve(torch_cuda, case):
    from oracle.solver import Reduced
    torch = torch_cuda
    pb = _te(inputs.tiny_m4() if case == "tiny" else inputs.small(12, 6, seed=21))
    red = Reduced(pb)
    G = red.G
    ctx = _ctx(pb)
    check_orders(ctx.get_mie(), red.s, np.ones(G.n_beta), G.P, 1e-11, tag=f"TE {case} Mie")
    A, E = ctx.get_A()
    assert np.max(np.abs(E / red.pinv.E - 1)) < 1e-12
    assert np.max(np.abs(A - red.A * red.pinv.E[None, :])) < 1e-12
    xh = probe(pb, 3)
    xd = torch.tensor(xh, dtype=torch.complex128, device="cuda:0")
    D = dscale(pb)
    check_orders(_np(ctx.apply_T(xd)), red.T_apply(xh), D, G.P, 1e-12, tag=f"TE {case} T")
    check_orders(_np(ctx.apply_lowrank(xd)), red.lowrank_apply(xh), D, G.P, 1e-9,
                 tag=f"TE {case} lowrank")
    check_orders(_np(ctx.apply(xd)), red.K_apply(xh), D, G.P, 1e-9, tag=f"TE {case} K")
    check_orders(_np(ctx.rhs()), red.rhs(), D, G.P, 1e-9, 1e-12, tag=f"TE {case} rhs")
    beta_o = red.solve_lu()
    oo = red.bragg(beta_o)
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    for kw in ({}, {"precision": GRT_FP32_RELAXED}):
        beta, st = ctx.solve(tol=1e-12, restart=150, **kw)
        say(f"[gpu] TE {case} {kw}: iters={st.iters} resid={st.rel_resid:.2e}")
        assert st.rel_resid <= 1e-12
        check_orders(_np(beta), beta_o, D, G.P, 1e-9, 1e-10, tag=f"TE {case} beta {kw}")
        og = ctx.bragg(beta)
        _bragg(og, oo, f"TE {case} Bragg")
        assert og["flux_err"] < 1e-10
    ctx.close()


def test_te_batch_mixes_polarisations(torch_cuda):
    """A lockstep batch of TE and TM problems reaches each one's oracle solution
    (the TE factors live in each context's own layer factors)."""
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Batch
    pbs = [_te(inputs.small(12, 6, seed=21)), inputs.small(12, 6, seed=21),
           _te(inputs.small(20, 10, seed=8, phi=0.3))]
    ctxs = [_ctx(pb) for pb in pbs]
    batch = Batch(ctxs)
    betas, stats = batch.solve(tol=1e-12, restart=150)
    for pb, b, st in zip(pbs, betas, stats):
        assert st.rel_resid <= 1e-12
        check_orders(_np(b), Reduced(pb).solve_lu(), dscale(pb), pb.P, 1e-9, 1e-10,
                     tag=f"TE batch {pb.name} {pb.polarization}")
    batch.close()
    for c in ctxs:
        c.close()


def test_te_refused_where_unsupported(torch_cuda):
    from paper_1412_7466_amd.grating import Context, GratingError, GRT_EUNSUP
    pb = _te(inputs.small(6, 6, seed=3))
    ctx = _ctx(pb)
    with pytest.raises(GratingError) as ei:
        ctx.eval_field(ctx.new_vec(), np.zeros((1, 2)))
    assert ei.value.status == GRT_EUNSUP
    st = _te(inputs.star(8, 6, seed=12))
    c2 = Context(0)
    with pytest.raises(GratingError) as ei:
        c2.set_problem(st)
    assert ei.value.status == GRT_EUNSUP
    c2.close()
    ctx.close()
