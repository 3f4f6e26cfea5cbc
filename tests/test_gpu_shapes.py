"""Non-circular inclusions on the GPU (paper sec. 4.1, eqs. intg1, intg2 and the
s_ln formula; shapes of eq. par1) against the CPU oracle (oracle/inclusion.py,
pinned in tests/test_oracle_inclusion.py).

The library solves each inclusion's integral equation at build time (batched LU on
the device) and applies the dense block-diagonal scattering matrix in every apply.
Bars: the scattering-matrix blocks to 1e-12 of each block's largest entry (both
sides solve the same discretisation); K per order to 1e-9, the mixed apply to 1e-4;
solutions per order to 1e-9 (plus 1e-10 of the largest order), the propagating Bragg
amplitudes to 1e-9 and the flux to 1e-9.
"""
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


def _ctx(pb):
    from paper_1412_7466_amd.grating import Context
    say(f"[gpu] shapes case {pb.name} M={pb.M} P={pb.P} nodes={pb.shape_nodes}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return ctx


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("M,P,seed,nodes", [(12, 8, 9, 64), (30, 10, 10, 48), (20, 15, 11, 96)])
def test_scattering_blocks_match_oracle(torch_cuda, M, P, seed, nodes):
    from oracle.inclusion import scattering_matrix
    pb = inputs.star(M, P, seed=seed, shape_nodes=nodes)
    ctx = _ctx(pb)
    Sg = _np(ctx.scattering_blocks())
    k2 = pb.omega * pb.n_layer[1]
    worst = 0.0
    for m in range(M):
        a1, a2, a3, rot = pb.shape[m]
        So = scattering_matrix(a1, a2, a3, rot, k2, pb.omega * pb.n_incl[m], P, n=nodes // 2)
        worst = max(worst, np.abs(Sg[m] - So).max() / np.abs(So).max())
    say(f"[gpu] {pb.name}: worst block error {worst:.2e}")
    assert worst <= 1e-12
    ctx.close()


def test_disk_blocks_are_mie(torch_cuda):
    from oracle.multiple import mie_coefficients
    pb = inputs.small(10, 6, seed=3)
    ctx = _ctx(pb)
    Sg = _np(ctx.scattering_blocks())
    m = mie_coefficients(pb.omega * pb.n_layer[1], pb.omega * np.asarray(pb.n_incl),
                         np.asarray(pb.radius), pb.P)
    for j in range(pb.M):
        assert np.abs(Sg[j] - np.diag(m[j])).max() <= 1e-12 * np.abs(m[j]).max()
    ctx.close()


@pytest.mark.parametrize("M,P,seed", [(12, 8, 9), (30, 10, 10)])
def test_shapes_apply_and_solve(torch_cuda, M, P, seed):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import GRT_FP32, GRT_FP32_RELAXED
    torch = torch_cuda
    pb = inputs.star(M, P, seed=seed)
    red = Reduced(pb)
    ctx = _ctx(pb)
    D = dscale(pb)
    xh = probe(pb, seed)
    xd = torch.tensor(xh, dtype=torch.complex128, device="cuda:0")
    y = _np(ctx.apply(xd))
    check_orders(y, red.K_apply(xh), D, P, 1e-9, tag=f"{pb.name} K probe")
    y32 = _np(ctx.apply(xd, precision=GRT_FP32))
    check_orders(y32, y, D, P, 1e-4, tag=f"{pb.name} mixed apply vs FP64")
    check_orders(_np(ctx.rhs()), red.rhs(), D, P, 1e-9, tag=f"{pb.name} rhs")
    beta_o = red.solve_lu()
    oo = red.bragg(beta_o)
    for prec in (None, GRT_FP32_RELAXED, GRT_FP32):
        kw = {} if prec is None else {"precision": prec}
        beta, st = ctx.solve(tol=1e-12, restart=150, **kw)
        say(f"[gpu] {pb.name} precision {prec}: iters={st.iters} resid={st.rel_resid:.2e}")
        assert st.rel_resid <= 1e-12
        check_orders(_np(beta), beta_o, D, P, 1e-9, 1e-10, tag=f"{pb.name} beta {prec}")
        og = ctx.bragg(beta)
        vg = np.concatenate([og["c"][oo["prop1"]], og["d"][oo["prop3"]]])
        vo = np.concatenate([oo["c"][oo["prop1"]], oo["d"][oo["prop3"]]])
        check_amplitudes(vg, vo, 1e-9, tag=f"{pb.name} Bragg {prec}")
        assert og["flux_err"] < 1e-9
    ctx.close()


def test_circles_as_shapes_match_disks(torch_cuda):
    """Disks entered as shapes (a2 = 0, turned) go through the dense path and give
    the disk path's solution."""
    pb = inputs.small(12, 6, seed=21)
    ctx = _ctx(pb)
    b0, _ = ctx.solve(tol=1e-13, restart=150)
    pb2 = inputs.small(12, 6, seed=21)
    pb2.shape = np.stack([pb2.radius, 0 * pb2.radius, np.full(12, 3.0),
                          np.linspace(0.0, 1.0, 12)], axis=1)
    ctx2 = _ctx(pb2)
    b2, _ = ctx2.solve(tol=1e-13, restart=150)
    check_orders(_np(b2), _np(b0), dscale(pb), pb.P, 1e-11, 1e-12, tag="circles as shapes")
    ctx.close()
    ctx2.close()


def test_batched_shapes_and_disks(torch_cuda):
    """A lockstep batch of non-circular and disk problems (FP64, relaxed mixed with an
    FP32 table on one of them, refinement mixed) reaches every problem's oracle
    solution."""
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Batch, GRT_FP32, GRT_FP32_RELAXED
    pbs = [inputs.star(12, 8, seed=9), inputs.small(20, 10, seed=25),
           inputs.star(30, 10, seed=10, phi=0.3), inputs.star(5, 6, seed=13)]
    ctxs = [_ctx(pb) for pb in pbs]
    ctxs[2].set_table32(True)
    refs = [Reduced(pb).solve_lu() for pb in pbs]
    batch = Batch(ctxs)
    for prec in (None, GRT_FP32_RELAXED, GRT_FP32):
        kw = {} if prec is None else {"precision": prec, "inner_tol": 1e-4 if prec == 2 else 0.0}
        betas, stats = batch.solve(tol=1e-12, restart=150, graph=True, **kw)
        for pb, b, st, ref in zip(pbs, betas, stats, refs):
            say(f"[gpu] batch {pb.name} precision {prec}: iters={st.iters} resid={st.rel_resid:.2e}")
            assert st.rel_resid <= 1e-12
            check_orders(_np(b), ref, dscale(pb), pb.P, 1e-9, 1e-10,
                         tag=f"batch {pb.name} {prec}")
    batch.close()
    for c in ctxs:
        c.close()


def test_shapes_refused_where_unsupported(torch_cuda):
    from paper_1412_7466_amd.grating import Context, GratingError, GRT_EINVAL, GRT_EUNSUP
    pb = inputs.star(8, 6, seed=12)
    ctx = _ctx(pb)
    with pytest.raises(GratingError) as ei:
        ctx.eval_field(ctx.new_vec(), np.zeros((1, 2)))
    assert ei.value.status == GRT_EUNSUP
    with pytest.raises(GratingError) as ei:
        ctx.apply_ST_block(ctx.new_vec())
    assert ei.value.status == GRT_EUNSUP
    # several angles, and shapes whose radius is not the enclosing circle
    c2 = Context(0)
    with pytest.raises(GratingError) as ei:
        c2.set_problem(pb, phis=[-0.3, 0.2])
    assert ei.value.status == GRT_EUNSUP
    bad = inputs.star(8, 6, seed=12)
    bad.radius = bad.radius * 1.01
    with pytest.raises(GratingError) as ei:
        c2.set_problem(bad)
    assert ei.value.status == GRT_EINVAL
    c2.close()
    ctx.close()
