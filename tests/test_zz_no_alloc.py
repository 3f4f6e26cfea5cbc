"""grt_apply_T_noalloc (the translation without a context or allocation) against the
context entry point grt_apply_T and the CPU FP64 oracle, on two calls in a row, the
second with a smaller problem (the scratch array keeps the first call's contents)."""
import cmath
import math

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from parity import check_orders, dscale, probe

pytestmark = pytest.mark.gpu


def _run(torch, pb, seed):
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Context, apply_T_noalloc
    print(f"[gpu] noalloc case {pb.name} M={pb.M} P={pb.P}", flush=True)
    xh = probe(pb, seed)
    dev = torch.device("cuda:0")
    x = torch.tensor(xh, dtype=torch.complex128, device=dev)
    cx = torch.tensor(np.asarray(pb.x, float), device=dev)
    cy = torch.tensor(np.asarray(pb.y, float), device=dev)
    k1, k2 = pb.omega * pb.n_layer[0], pb.omega * pb.n_layer[1]
    alpha = cmath.exp(1j * k1 * math.sin(pb.phi) * pb.d)
    y = torch.full_like(x, complex(float("nan"), float("nan")))
    apply_T_noalloc(pb.P, k2, pb.d, alpha, cx, cy, x, y)
    torch.cuda.synchronize()
    y_na = y.cpu().numpy()
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    y_ctx = ctx.apply_T(x).cpu().numpy()
    ctx.close()
    D = dscale(pb)
    check_orders(y_na, y_ctx, D, pb.P, 1e-13, tag=f"{pb.name} noalloc vs grt_apply_T")
    check_orders(y_na, Reduced(pb).T_apply(xh), D, pb.P, 1e-12, tag=f"{pb.name} noalloc vs oracle")


def test_noalloc_matches_context_apply_T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    _run(torch, inputs.small(150, 10, seed=16), 1)
    _run(torch, inputs.small(13, 6, seed=5, phi=0.3), 2)


def test_noalloc_rejects_bad_input():
    import torch
    from paper_1412_7466_amd.grating import GRT_EINVAL, GRT_EUNSUP, GratingError, apply_T_noalloc
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    dev = torch.device("cuda:0")
    cx = torch.zeros(3, dtype=torch.float64, device=dev)
    x = torch.zeros(3 * 15, dtype=torch.complex128, device=dev)
    y = torch.zeros_like(x)
    with pytest.raises(GratingError) as ei:
        apply_T_noalloc(7, 10.0, 1.0, 1.0 + 0j, cx, cx, x, y)       # P not compiled in
    assert ei.value.status == GRT_EUNSUP
    with pytest.raises(GratingError) as ei:
        apply_T_noalloc(7, 10.0, 1.0, 2.0 + 0j, cx, cx, x, y)       # |alpha| != 1
    assert ei.value.status == GRT_EINVAL
    # M (2P+1) beyond one partial result of the 64 MiB scratch: refused on the host
    big = 4_194_304 // 41 + 1
    cxb = torch.zeros(big, dtype=torch.float64, device=dev)
    xb = torch.zeros(big * 41, dtype=torch.complex128, device=dev)
    with pytest.raises(GratingError) as ei:
        apply_T_noalloc(20, 10.0, 1.0, 1.0 + 0j, cxb, cxb, xb, torch.zeros_like(xb))
    assert ei.value.status == GRT_EINVAL
