"""An absorbing substrate on the GPU (bottom layer index n_3 + i n3_im, TM and TE) against
the CPU oracle's (pinned in tests/test_oracle_substrate.py: the Fresnel slab with
complex k_3 and its energy balance, independence of the artificial line Gamma_d).

The library assembles the layer matrix with H_0, H_1 and J_n at complex arguments
(checked on the host in tests/test_device_math_cpu.py) and the Rayleigh-Bloch
wavenumbers k_3n on the decaying branch (TE: the substrate's factors eps_3 and 1/eps_3
complex); the apply kernels are unchanged.  Bars as for
the lossless layers: equilibrated A to 1e-12, K, the right-hand side, solutions and
Bragg amplitudes 1e-9; the transmitted powers 1e-9 relative.
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


def _ctx(pb):
    from paper_1412_7466_amd.grating import Context
    say(f"[gpu] substrate case {pb.name} M={pb.M} P={pb.P} n3_im={pb.n3_im}")
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
    assert math.isnan(og["flux_err"])
    sel = oo["prop3"]
    assert np.max(np.abs(og["T"][sel] - oo["T"][sel])) < 1e-9 * max(oo["T"][sel].sum(), 1e-3)


@pytest.mark.parametrize("phi,n3_im,pol", [(-math.pi / 5, 0.05, "TM"), (0.3, 0.12, "TM"),
                                           (0.3, 0.12, "TE")])
def test_substrate_empty_slab(torch_cuda, phi, n3_im, pol):
    from oracle.solver import Reduced
    pb = inputs.empty_slab(phi=phi)
    pb.n3_im = n3_im
    pb.polarization = pol
    red = Reduced(pb)
    ctx = _ctx(pb)
    og = ctx.bragg()
    oo = red.bragg(np.zeros(0))
    i0 = list(oo["orders"]).index(0)
    assert abs(og["c"][i0] - oo["c"][i0]) < 1e-12
    assert abs(og["d"][i0] - oo["d"][i0]) < 1e-12
    assert abs(og["T"][i0] - oo["T"][i0]) < 1e-12
    assert math.isnan(og["flux_err"])
    ctx.close()


@pytest.mark.parametrize("case", ["flat", "curved", "absorbing_disks", "te", "te_curved"])
def test_substrate_pieces_and_solve(torch_cuda, case):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    torch = torch_cuda
    if case == "absorbing_disks":
        pb = inputs.lossy(12, 6, seed=21)
        pb.n3_im = 0.08
    else:
        pb = inputs.lossy_substrate(12, 6, seed=21, n3_im=0.08, curved_iface=case.endswith("curved"))
        if case.startswith("te"):
            pb.polarization = "TE"
    red = Reduced(pb)
    G = red.G
    ctx = _ctx(pb)
    A, E = ctx.get_A()
    assert np.max(np.abs(E / red.pinv.E - 1)) < 1e-12
    assert np.max(np.abs(A - red.A * red.pinv.E[None, :])) < 1e-12
    xh = probe(pb, 3)
    xd = torch.tensor(xh, dtype=torch.complex128, device="cuda:0")
    D = dscale(pb)
    check_orders(_np(ctx.apply_lowrank(xd)), red.lowrank_apply(xh), D, G.P, 1e-9,
                 tag=f"substrate {case} lowrank")
    check_orders(_np(ctx.apply(xd)), red.K_apply(xh), D, G.P, 1e-9, tag=f"substrate {case} K")
    check_orders(_np(ctx.rhs()), red.rhs(), D, G.P, 1e-9, 1e-12, tag=f"substrate {case} rhs")
    beta_o = red.solve_lu()
    oo = red.bragg(beta_o)
    for kw in ({}, {"precision": GRT_FP32_RELAXED}):
        beta, st = ctx.solve(tol=1e-12, restart=150, **kw)
        say(f"[gpu] substrate {case} {kw}: iters={st.iters} resid={st.rel_resid:.2e}")
        assert st.rel_resid <= 1e-12
        check_orders(_np(beta), beta_o, D, G.P, 1e-9, 1e-10, tag=f"substrate {case} beta {kw}")
        og = ctx.bragg(beta)
        _bragg(og, oo, f"substrate {case} Bragg")
        if case == "absorbing_disks":
            assert abs(og["absorbed"] - oo["absorbed"]) < 1e-9 * oo["absorbed"]
    ctx.close()


def test_substrate_does_not_share_lossless_factors(torch_cuda):
    """The layer factors are shared between contexts with equal layers: the loss is
    part of what makes them equal."""
    from oracle.solver import Reduced
    a = inputs.small(8, 6, seed=4)
    b = inputs.lossy_substrate(8, 6, seed=4, n3_im=0.05)
    ca, cb = _ctx(a), _ctx(b)
    for pb, ctx in ((a, ca), (b, cb)):
        beta, st = ctx.solve(tol=1e-12, restart=150)
        check_orders(_np(beta), Reduced(pb).solve_lu(), dscale(pb), pb.P, 1e-9, 1e-10,
                     tag=f"shared factors {pb.name}")
    ca.close()
    cb.close()


def test_substrate_batch(torch_cuda):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Batch
    pbs = [inputs.lossy_substrate(12, 6, seed=21, n3_im=0.08), inputs.small(12, 6, seed=21)]
    ctxs = [_ctx(pb) for pb in pbs]
    batch = Batch(ctxs)
    betas, stats = batch.solve(tol=1e-12, restart=150)
    for pb, b, s in zip(pbs, betas, stats):
        assert s.rel_resid <= 1e-12
        check_orders(_np(b), Reduced(pb).solve_lu(), dscale(pb), pb.P, 1e-9, 1e-10,
                     tag=f"substrate batch {pb.name}")
    batch.close()
    for c in ctxs:
        c.close()


def test_substrate_refused_where_unsupported(torch_cuda):
    from paper_1412_7466_amd.grating import Context, GratingError, GRT_EINVAL, GRT_EUNSUP
    pb = inputs.lossy_substrate(6, 6, seed=3, n3_im=0.05)
    ctx = _ctx(pb)
    with pytest.raises(GratingError) as ei:
        ctx.eval_field(ctx.new_vec(), np.zeros((1, 2)))
    assert ei.value.status == GRT_EUNSUP
    ctx.close()
    c2 = Context(0)
    for n3_im, pol, status in ((-0.01, "TM", GRT_EINVAL), (0.5, "TM", GRT_EUNSUP),
                               (0.5, "TE", GRT_EUNSUP)):
        bad = inputs.lossy_substrate(6, 6, seed=3, n3_im=n3_im)
        bad.polarization = pol
        with pytest.raises(GratingError) as ei:
            c2.set_problem(bad)
        assert ei.value.status == status
    c2.close()
