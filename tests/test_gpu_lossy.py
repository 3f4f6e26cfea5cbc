"""Absorbing disks on the GPU (complex inclusion index n + i n_im) against the CPU
oracle's absorbing disks (pinned in tests/test_oracle_lossy.py: interface conditions
of the Mie coefficients at complex argument, energy balance R + T + absorbed = 1).

The library computes the Mie coefficients at the complex interior argument k_p R
(Miller's recurrence, checked on the host in tests/test_device_math_cpu.py); the rest
of the path is the lossless one.  Bars: the Mie diagonal per order 1e-11, solutions
and Bragg amplitudes 1e-9, the absorbed fraction 1e-9 relative, the energy balance
1e-10.
"""
import sys

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from parity import check_amplitudes, check_orders, dscale

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


def _ctx(pb):
    from paper_1412_7466_amd.grating import Context
    say(f"[gpu] lossy case {pb.name} M={pb.M} P={pb.P} pol={pb.polarization}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return ctx


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_lossy_mie_solve_and_energy(torch_cuda, pol):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    pb = inputs.lossy(12, 8, seed=21)
    pb.polarization = pol
    red = Reduced(pb)
    G = red.G
    ctx = _ctx(pb)
    check_orders(ctx.get_mie(), red.s, np.ones(G.n_beta), G.P, 1e-11, tag=f"lossy {pol} Mie")
    D = dscale(pb)
    beta_o = red.solve_lu()
    oo = red.bragg(beta_o)
    for kw in ({}, {"precision": GRT_FP32_RELAXED}):
        beta, st = ctx.solve(tol=1e-12, restart=150, **kw)
        say(f"[gpu] lossy {pol} {kw}: iters={st.iters} resid={st.rel_resid:.2e}")
        assert st.rel_resid <= 1e-12
        check_orders(_np(beta), beta_o, D, G.P, 1e-9, 1e-10, tag=f"lossy {pol} beta {kw}")
        og = ctx.bragg(beta)
        vg = np.concatenate([og["c"][oo["prop1"]], og["d"][oo["prop3"]]])
        vo = np.concatenate([oo["c"][oo["prop1"]], oo["d"][oo["prop3"]]])
        check_amplitudes(vg, vo, 1e-9, tag=f"lossy {pol} Bragg")
        say(f"[gpu] lossy {pol}: absorbed {og['absorbed']:.6f} (oracle {oo['absorbed']:.6f}), "
            f"balance error {og['flux_err']:.1e}")
        assert abs(og["absorbed"] - oo["absorbed"]) < 1e-9 * oo["absorbed"]
        assert og["absorbed"] > 0.05
        assert og["flux_err"] < 1e-10
    ctx.close()


def test_lossy_batch_with_lossless(torch_cuda):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Batch
    pbs = [inputs.lossy(12, 8, seed=21), inputs.small(12, 8, seed=21),
           inputs.lossy(20, 10, seed=8, phi=0.3, loss=(0.01, 0.1))]
    ctxs = [_ctx(pb) for pb in pbs]
    batch = Batch(ctxs)
    betas, stats = batch.solve(tol=1e-12, restart=150)
    for pb, b, s in zip(pbs, betas, stats):
        assert s.rel_resid <= 1e-12
        check_orders(_np(b), Reduced(pb).solve_lu(), dscale(pb), pb.P, 1e-9, 1e-10,
                     tag=f"lossy batch {pb.name}")
    batch.close()
    for c in ctxs:
        c.close()


def test_lossy_refused_where_unsupported(torch_cuda):
    from paper_1412_7466_amd.grating import Context, GratingError, GRT_EINVAL, GRT_EUNSUP
    pb = inputs.lossy(6, 6, seed=3)
    ctx = _ctx(pb)
    with pytest.raises(GratingError) as ei:
        ctx.eval_field(ctx.new_vec(), np.zeros((1, 2)))
    assert ei.value.status == GRT_EUNSUP
    ctx.close()
    c2 = Context(0)
    bad = inputs.lossy(6, 6, seed=3)
    bad.n_incl_im = -bad.n_incl_im
    with pytest.raises(GratingError) as ei:
        c2.set_problem(bad)
    assert ei.value.status == GRT_EINVAL
    far = inputs.lossy(6, 6, seed=3)
    far.n_incl_im = np.full(6, 10.0)       # Im(k_p R) = 10 * 10 * R > 2 for R >= 0.02
    with pytest.raises(GratingError) as ei:
        c2.set_problem(far)
    assert ei.value.status == GRT_EUNSUP
    st = inputs.star(8, 6, seed=12)
    st.n_incl_im = np.full(8, 0.1)
    with pytest.raises(GratingError) as ei:
        c2.set_problem(st)
    assert ei.value.status == GRT_EUNSUP
    c2.close()
