"""Several right-hand sides (incidence angles) on one geometry (grt_incidence n_rhs /
phis): the block translation on the FP32 matrix cores against the oracle, the
stacked applies, the lockstep solves in FP64 and with FP32 block translation plus
FP64 refinement, and the per-angle Bragg amplitudes and fields.

Bars (per order in the normalised basis, tests/parity.py): S T and K through the FP32
block product 1e-5 of each order plus 1e-6 of the largest (FP32 arithmetic; at
M = 10000 the bar grows with the square root of the accumulation length);
FP64 applies 1e-9; solutions 1e-9 plus 1e-10 of the largest order; Bragg amplitudes
1e-9 each."""
import dataclasses
import math

import numpy as np
import pytest

from paper_1412_7466_amd import inputs
from parity import check_amplitudes, check_orders, dscale, probe

pytestmark = pytest.mark.gpu


def _case(M, P, seed, R, omega=10.0):
    pb0 = inputs.small(M, P, omega=omega, seed=seed)
    phis = list(np.linspace(-math.pi / 3, math.pi / 3, R))
    return pb0, phis, [dataclasses.replace(pb0, phi=float(p)) for p in phis]


def _ctx(pb0, phis):
    from paper_1412_7466_amd.grating import Context
    print(f"[gpu] block case M={pb0.M} P={pb0.P} R={len(phis)}", flush=True)
    import time
    ctx = Context(0)
    ctx.set_problem(pb0, phis=phis)
    t0 = time.perf_counter()
    ctx.build()
    print(f"[gpu] block case built in {time.perf_counter() - t0:.1f} s", flush=True)
    assert ctx.n_rhs == len(phis)
    return ctx


def _oracle_ST_rows(pb, phi, x, rows):
    """s_j (T x)_j for the target rows, by the oracle at angle phi (no layered
    structure needed)."""
    from oracle.common import Geometry
    from oracle.multiple import apply_T_rows, mie_coefficients
    G = Geometry(dataclasses.replace(pb, phi=float(phi)))
    s = mie_coefficients(G.k2, G.kp[rows], G.rad[rows], G.P)
    return (s * apply_T_rows(G, x, rows)).reshape(-1)


def _block_ctx(pb, phis):
    import time
    from paper_1412_7466_amd.grating import Context
    print(f"[gpu] large block M={pb.M} P={pb.P} R={len(phis)} (translation only)", flush=True)
    ctx = Context(0)
    ctx.set_problem(pb, phis=list(phis))
    t0 = time.perf_counter()
    ctx.build_translation()
    print(f"[gpu] translation data built in {time.perf_counter() - t0:.1f} s", flush=True)
    return ctx


@pytest.mark.parametrize("M,P,seed,R", [(30, 10, 41, 5), (25, 20, 14, 3), (40, 4, 42, 65)])
def test_block_translation_matches_oracle(M, P, seed, R):
    """y_r = S T_r x_r for every angle at once on the FP32 matrix cores (one work-group
    column tile for R <= 64, two for R = 65), against the oracle per angle; the
    context is built for the translation only."""
    import torch
    pb0, phis, pbs = _case(M, P, seed, R)
    ctx = _block_ctx(pb0, phis)
    D = dscale(pb0)
    xs = [probe(pb0, 100 + r) for r in range(R)]
    x = torch.tensor(np.concatenate(xs), dtype=torch.complex128, device="cuda:0")
    y = ctx.apply_ST_block(x).cpu().numpy().reshape(R, -1)
    rows = np.arange(M)
    check_r = range(R) if R <= 8 else (0, 1, 33, 63, 64)
    for r in check_r:
        ref = _oracle_ST_rows(pb0, phis[r], xs[r], rows)
        check_orders(y[r], ref, D, P, 1e-5, 1e-6, tag=f"block S T angle {r}")
    ctx.close()


def test_block_applies_match_oracle():
    """K of every angle: FP64 (per-angle kernels) to 1e-9 per order, FP32 (block
    translation, FP64 layer correction) to the FP32 bar; T and the right-hand side."""
    import torch
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import GRT_FP32
    pb0, phis, pbs = _case(30, 10, 41, 4)
    ctx = _ctx(pb0, phis)
    R = len(phis)
    D = dscale(pb0)
    xs = [probe(pb0, 200 + r) for r in range(R)]
    x = torch.tensor(np.concatenate(xs), dtype=torch.complex128, device="cuda:0")
    y64 = ctx.apply(x).cpu().numpy().reshape(R, -1)
    y32 = ctx.apply(x, precision=GRT_FP32).cpu().numpy().reshape(R, -1)
    yT = ctx.apply_T(x).cpu().numpy().reshape(R, -1)
    b = ctx.rhs().cpu().numpy().reshape(R, -1)
    for r in range(R):
        red = Reduced(pbs[r])
        K = red.K_apply(xs[r])
        check_orders(y64[r], K, D, 10, 1e-9, tag=f"block K FP64 angle {r}")
        check_orders(y32[r], K, D, 10, 1e-5, 1e-6, tag=f"block K FP32 angle {r}")
        check_orders(yT[r], red.T_apply(xs[r]), D, 10, 1e-12, tag=f"block T angle {r}")
        check_orders(b[r], red.rhs(), D, 10, 1e-9, 1e-12, tag=f"block rhs angle {r}")
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_block_solves_match_oracle(precision):
    """All angles solved together (one lockstep batch; FP32: block translation inside
    FP64 refinement) reach each angle's oracle LU solution; Bragg amplitudes and the
    field per angle."""
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import GRT_FP32, GRT_FP64
    pb0, phis, pbs = _case(30, 10, 41, 4)
    ctx = _ctx(pb0, phis)
    R = len(phis)
    prec = GRT_FP32 if precision == "fp32" else GRT_FP64
    beta, stats = ctx.solve(tol=1e-12, restart=150, precision=prec, inner_tol=1e-5)
    assert len(stats) == R
    bh = beta.cpu().numpy().reshape(R, -1)
    D = dscale(pb0)
    for r in range(R):
        red = Reduced(pbs[r])
        bo = red.solve_lu()
        print(f"[gpu] block {precision} angle {r}: iters {stats[r].iters} refine "
              f"{stats[r].refine_steps} resid {stats[r].rel_resid:.2e}", flush=True)
        assert stats[r].rel_resid <= 1e-12
        check_orders(bh[r], bo, D, 10, 1e-9, 1e-10, tag=f"block solve {precision} angle {r}")
        og = ctx.bragg(beta[r * ctx.sizes.n_beta:(r + 1) * ctx.sizes.n_beta], rhs=r)
        oo = red.bragg(bo)
        vg = np.concatenate([og["c"][oo["prop1"]], og["d"][oo["prop3"]]])
        vo = np.concatenate([oo["c"][oo["prop1"]], oo["d"][oo["prop3"]]])
        check_amplitudes(vg, vo, 1e-9, tag=f"block Bragg angle {r}")
        assert og["flux_err"] < 1e-9
        if precision == "fp64" and r in (0, R - 1):
            xy = np.array([[0.1, 0.8], [-0.3, 0.1], [0.45, -0.9]])
            u = ctx.eval_field(beta[r * ctx.sizes.n_beta:(r + 1) * ctx.sizes.n_beta], xy, rhs=r)
            from oracle.field import Field
            uo = Field(red, bo).total(xy[:, 0], xy[:, 1])
            assert np.max(np.abs(u - uo)) < 1e-9 * np.max(np.abs(uo))
    ctx.close()


def test_multi_rhs_rejected_where_unsupported():
    from paper_1412_7466_amd.grating import Batch, GratingError, GRT_EINVAL
    pb0, phis, _ = _case(5, 4, 43, 2)
    ctx = _ctx(pb0, phis)
    with pytest.raises(GratingError) as ei:
        Batch([ctx])
    assert ei.value.status == GRT_EINVAL
    with pytest.raises(GratingError) as ei:
        ctx.bragg(ctx.new_vec(one=True), rhs=2)
    assert ei.value.status == GRT_EINVAL
    ctx.close()


def test_block_large_shape_reduced_M():
    """The large block geometry's rules (d=4, omega=40, P=20, 16 angles) at M=300:
    every angle and target against the oracle."""
    import torch
    pb, phis = inputs.large_block(M=300, R=16)
    ctx = _block_ctx(pb, phis)
    R = len(phis)
    D = dscale(pb)
    xs = [probe(pb, 300 + r) for r in range(R)]
    x = torch.tensor(np.concatenate(xs), dtype=torch.complex128, device="cuda:0")
    y = ctx.apply_ST_block(x).cpu().numpy().reshape(R, -1)
    rows = np.arange(pb.M)
    for r in range(R):
        ref = _oracle_ST_rows(pb, phis[r], xs[r], rows)
        check_orders(y[r], ref, D, pb.P, 1e-5, 1e-6, tag=f"large shape M=300 angle {r}")
    from paper_1412_7466_amd.grating import GratingError, GRT_ESTATE
    with pytest.raises(GratingError) as ei:
        ctx.apply(x)                      # the layered structure is not built
    assert ei.value.status == GRT_ESTATE
    ctx.close()


def test_block_full_size_sampled():
    """M=10000, P=20, 256 angles, the launch configuration the benchmark times: sampled
    targets of sampled angles against the oracle, one by one."""
    import torch
    pb, phis = inputs.large_block()
    ctx = _block_ctx(pb, phis)
    R = len(phis)
    D = dscale(pb)
    rng = np.random.default_rng(11)
    u = rng.standard_normal((R, D.size)) + 1j * rng.standard_normal((R, D.size))
    x = torch.tensor((u / D[None, :]).reshape(-1), dtype=torch.complex128, device="cuda:0")
    del u
    y = ctx.apply_ST_block(x)
    torch.cuda.synchronize()
    nb = 2 * pb.P + 1
    rows = np.array([0, 1, 4097, 9998, 9999])
    sel = (rows[:, None] * nb + np.arange(nb)[None, :]).reshape(-1)
    # each output is one FP32 accumulator over 3 M ceil((2P+1)/4) = 3.3e5 MFMA steps: the
    # rounding of such a sum grows like sqrt(steps) u (u = 6e-8), 3.4e-5 of the terms'
    # size here, so the FP32 bar at this size is 3 sqrt(steps) u
    steps = 3 * pb.M * ((nb + 3) // 4)
    rtol = 3.0 * np.sqrt(steps) * 2.0 ** -24
    for r in (0, 63, 64, 255):
        xr = x[r * D.size:(r + 1) * D.size].cpu().numpy()
        yr = y[r * D.size:(r + 1) * D.size].cpu().numpy()[sel]
        ref = _oracle_ST_rows(pb, phis[r], xr, rows)
        check_orders(yr, ref, D[sel], pb.P, rtol, 1e-6, tag=f"full size angle {r}")
    ctx.close()
