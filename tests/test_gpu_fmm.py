"""The fast cell translation (grt_set_fmm) on the GPU.

Exact parity is against the CPU oracle's stored M=1000 results (tests/golden, from
oracle/ only): K on the stored probe, per order in the normalised basis, to the same
1e-9 as the dense translation, and the FP64 solution and Bragg amplitudes to 1e-9.
At larger M the cell translation is compared with the dense translation (itself
pinned to the oracle): S T on a probe, weighted D s per order (what enters K), to
1e-10 relative per order, at omega = 20 and 40 and P = 15, 20.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from parity import check_amplitudes, check_orders

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def test_fmm_m1000_against_oracle(torch_cuda):
    from paper_1412_7466_amd.grating import Context
    torch = torch_cuda
    pb = inputs.m1000()
    gold = np.load(os.path.join(GOLD, "m1000_oracle.npz"))
    assert str(gold["digest"]) == pb.digest()
    say(f"[gpu] fmm m1000 build")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    info = ctx.set_fmm(True)
    say(f"[gpu] fmm m1000 cells {info}")
    x = torch.tensor(gold["probe"], dtype=torch.complex128, device="cuda:0")
    D = gold["D"]
    check_orders(ctx.apply(x).cpu().numpy(), gold["K_probe"], D, pb.P, 1e-9,
                 tag="fmm m1000 K probe")
    beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
    say(f"[gpu] fmm m1000 iters={st.iters} resid={st.rel_resid:.2e}")
    assert st.rel_resid <= 1e-12
    check_orders(beta.cpu().numpy(), gold["beta"], D, pb.P, 1e-9, 1e-10, tag="fmm m1000 beta")
    og = ctx.bragg(beta)
    p1, p3 = gold["prop1"], gold["prop3"]
    check_amplitudes(np.concatenate([og["c"][p1], og["d"][p3]]),
                     np.concatenate([gold["c"][p1], gold["d"][p3]]), 1e-9, tag="fmm m1000 Bragg")
    # and back to the dense translation: the same operator again
    ctx.set_fmm(False)
    check_orders(ctx.apply(x).cpu().numpy(), gold["K_probe"], D, pb.P, 1e-9,
                 tag="dense again K probe")
    ctx.close()


@pytest.mark.parametrize("M,omega,P,per_cell,bar", [(3000, 20.0, 15, 40, 1e-10),
                                                    (6000, 40.0, 20, 40, 1e-10),
                                                    (2000, 40.0, 20, 16, 1e-10),
                                                    (20000, 40.0, 20, 0, 1e-12)])
def test_fmm_matches_dense_translation(torch_cuda, M, omega, P, per_cell, bar):
    """Translation-only builds of the large block geometry (d = 4, middle layer
    [-2, 2]) at M inclusions: S T x by cells against the dense S T x.  per_cell 0: the
    default cells, which must hold 1e-12 per order also at M = 20000 (16 per cell
    there would give cells with k s sqrt 2 < 10 and about 1e-11)."""
    from paper_1412_7466_amd.grating import Context
    torch = torch_cuda
    pb = inputs.make_problem(f"fmm_M{M}", 4.0, 2.0, M, 0.005, 0.01, 1.5, 3.0, 0.002, 4, omega,
                             -math.pi / 5, P)
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build_translation()
    s = ctx.get_mie()
    k2 = omega * pb.n_layer[1]
    import scipy.special as sp
    n = np.abs(np.arange(-P, P + 1))
    D = np.abs(sp.hankel1(n[None, :], k2 * np.asarray(pb.radius)[:, None])).reshape(-1)
    rng = np.random.default_rng(M)
    u = rng.standard_normal(pb.M * (2 * P + 1)) + 1j * rng.standard_normal(pb.M * (2 * P + 1))
    x = torch.tensor(u / D, dtype=torch.complex128, device="cuda:0")
    y0 = ctx.apply_T(x).cpu().numpy()
    info = ctx.set_fmm(True, per_cell=per_cell)
    y1 = ctx.apply_T(x).cpu().numpy()
    say(f"[gpu] fmm M={M} omega={omega} P={P} cells {info}")
    check_orders(s * y1, s * y0, D, P, bar, tag=f"fmm M={M} S T")
    ctx.close()


def test_fmm_refused_where_unsupported(torch_cuda):
    from paper_1412_7466_amd.grating import (Batch, Context, GratingError, GRT_EUNSUP,
                                             GRT_FP32_RELAXED)
    pb = inputs.small(20, 6, seed=3)
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    ctx.set_fmm(True)
    with pytest.raises(GratingError) as ei:
        ctx.solve(tol=1e-10, precision=GRT_FP32_RELAXED)
    assert ei.value.status == GRT_EUNSUP
    with pytest.raises(GratingError) as ei:
        Batch([ctx])
    assert ei.value.status == GRT_EUNSUP
    ctx.close()
    c2 = Context(0)
    c2.set_problem(pb, phis=[-0.3, 0.2])
    c2.build_translation()
    with pytest.raises(GratingError) as ei:
        c2.set_fmm(True)
    assert ei.value.status == GRT_EUNSUP
    c2.close()


@pytest.mark.parametrize("case", ["star", "curved", "te", "lossy", "substrate"])
def test_fmm_with_other_features(torch_cuda, case):
    """The cell translation only replaces T: with non-circular inclusions, curved
    interfaces, TE, absorbing disks or an absorbing substrate the K apply and the
    solution stay those of the dense translation (1e-12 per order on K, 1e-10 on the
    solution)."""
    from paper_1412_7466_amd.grating import Context
    from parity import dscale, probe
    torch = torch_cuda
    pb = {"star": lambda: inputs.star(60, 8, seed=31),
          "curved": lambda: inputs.curved(60, 8, seed=32),
          "te": lambda: inputs.small(60, 8, seed=33),
          "lossy": lambda: inputs.lossy(60, 8, seed=34),
          "substrate": lambda: inputs.lossy_substrate(60, 8, seed=35, n3_im=0.08)}[case]()
    if case == "te":
        pb.polarization = "TE"
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    xh = probe(pb, 5)
    xd = torch.tensor(xh, dtype=torch.complex128, device="cuda:0")
    D = dscale(pb)
    y0 = ctx.apply(xd).cpu().numpy()
    b0, s0 = ctx.solve(tol=1e-12, restart=150)
    info = ctx.set_fmm(True, per_cell=8)
    say(f"[gpu] fmm {case}: cells {info}")
    check_orders(ctx.apply(xd).cpu().numpy(), y0, D, pb.P, 1e-12, tag=f"fmm {case} K")
    b1, s1 = ctx.solve(tol=1e-12, restart=150)
    check_orders(b1.cpu().numpy(), b0.cpu().numpy(), D, pb.P, 1e-10, 1e-11,
                 tag=f"fmm {case} beta")
    ctx.close()
