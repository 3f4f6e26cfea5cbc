"""Full-size parity: the M=1000 workload the benchmark times (P=15) and the same
geometry at P=20, against the CPU FP64 oracle's stored results
(tests/golden/m1000_oracle.npz, m1000_p20_oracle.npz, star_m1000_oracle.npz and
curved_m1000_oracle.npz, written by
tests/golden/make_m1000_oracle.py from oracle/ only).

Same launch configuration as the benchmark (the work split is a function of M and
the discretization only).  Every comparison is per order in the normalised basis
(tests/parity.py): T applied to the stored probe x = D^-1 u to 1e-12 of each order's
size, K to 1e-9; beta to 1e-9 per order plus 1e-10 of the largest order; each
propagating Bragg amplitude to 1e-9; flux error below 1e-9.
"""
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


def _load(case):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1412_7466_amd.grating import Context
    gold = np.load(os.path.join(GOLD, f"{case}_oracle.npz"))
    pb = getattr(inputs, case)()
    assert str(gold["digest"]) == pb.digest(), "inputs changed: regenerate the golden file"
    say(f"[gpu] {case} build M={pb.M} P={pb.P} N={pb.disc.N}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return torch, ctx, gold, pb


@pytest.fixture(scope="module")
def m1000():
    torch, ctx, gold, pb = _load("m1000")
    yield torch, ctx, gold, pb
    ctx.close()


def _check_apply(torch, ctx, gold, pb, tag):
    x = torch.tensor(gold["probe"], dtype=torch.complex128, device="cuda:0")
    D = gold["D"]
    yT = ctx.apply_T(x).cpu().numpy()
    check_orders(yT, gold["T_probe"], D, pb.P, 1e-12, tag=f"{tag} T probe")
    y = ctx.apply(x).cpu().numpy()
    check_orders(y, gold["K_probe"], D, pb.P, 1e-9, tag=f"{tag} K probe")


def _check_solution(ctx, beta, gold, pb, tag):
    check_orders(beta.cpu().numpy(), gold["beta"], gold["D"], pb.P, 1e-9, 1e-10,
                 tag=f"{tag} beta")
    og = ctx.bragg(beta)
    p1, p3 = gold["prop1"], gold["prop3"]
    vg = np.concatenate([og["c"][p1], og["d"][p3]])
    vo = np.concatenate([gold["c"][p1], gold["d"][p3]])
    check_amplitudes(vg, vo, 1e-9, tag=f"{tag} Bragg")
    say(f"[gpu] {tag}: flux {og['flux_err']:.2e}")
    assert og["flux_err"] < 1e-9


def test_m1000_apply(m1000):
    torch, ctx, gold, pb = m1000
    _check_apply(torch, ctx, gold, pb, "m1000")


def test_m1000_solve_fp64(m1000):
    torch, ctx, gold, pb = m1000
    beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
    say(f"[gpu] m1000 FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
    _check_solution(ctx, beta, gold, pb, "m1000 FP64")


def test_m1000_solve_mixed(m1000):
    from paper_1412_7466_amd.grating import GRT_FP32
    torch, ctx, gold, pb = m1000
    beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000, precision=GRT_FP32)
    say(f"[gpu] m1000 mixed iters={st.iters} refine={st.refine_steps} "
        f"resid={st.rel_resid:.2e} {st.seconds:.3f}s")
    _check_solution(ctx, beta, gold, pb, "m1000 mixed")


def test_m1000_solve_relaxed_fp32_table(m1000):
    """Relaxed mixed precision with the FP32 table of the well-separated pairs: FP64
    GMRES whose applies switch to the FP32 translation below 1e3 tol."""
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    torch, ctx, gold, pb = m1000
    ctx.set_table32(True)
    try:
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000, precision=GRT_FP32_RELAXED)
        say(f"[gpu] m1000 relaxed iters={st.iters} fp32 applies={st.fp32_applies} "
            f"resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        assert st.fp32_applies > 0
        _check_solution(ctx, beta, gold, pb, "m1000 relaxed")
    finally:
        ctx.set_table32(False)


def test_m1000_resident_table(m1000):
    """Same bars with the resident translation table (1 GB at this size)."""
    torch, ctx, gold, pb = m1000
    ctx.set_table(True)
    try:
        _check_apply(torch, ctx, gold, pb, "m1000 table")
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
        say(f"[gpu] m1000 table FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        _check_solution(ctx, beta, gold, pb, "m1000 FP64 table")
    finally:
        ctx.set_table(False)


def test_m1000_p20():
    """P=20 at M=1000: generator orders up to 40, the one-lane kernels' accumulators
    no longer fit in registers (split on-the-fly launch, two-lane table kernel)."""
    if not os.path.exists(os.path.join(GOLD, "m1000_p20_oracle.npz")):
        pytest.skip("tests/golden/m1000_p20_oracle.npz not generated")
    torch, ctx, gold, pb = _load("m1000_p20")
    try:
        _check_apply(torch, ctx, gold, pb, "m1000_p20")
        ctx.set_launch(16, 2)
        _check_apply(torch, ctx, gold, pb, "m1000_p20 split")
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
        say(f"[gpu] m1000_p20 FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        _check_solution(ctx, beta, gold, pb, "m1000_p20 FP64")
        ctx.set_table(2)
        _check_apply(torch, ctx, gold, pb, "m1000_p20 table 2 lanes")
    finally:
        ctx.close()


def test_star_m1000():
    """Non-circular inclusions (eq. par1) on the M=1000 packing: K and T on the stored
    probe, the FP64 and relaxed mixed solutions and their Bragg amplitudes against the
    oracle (tests/golden/star_m1000_oracle.npz)."""
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    if not os.path.exists(os.path.join(GOLD, "star_m1000_oracle.npz")):
        pytest.skip("tests/golden/star_m1000_oracle.npz not generated")
    torch, ctx, gold, pb = _load("star_m1000")
    try:
        _check_apply(torch, ctx, gold, pb, "star_m1000")
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
        say(f"[gpu] star_m1000 FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        _check_solution(ctx, beta, gold, pb, "star_m1000 FP64")
        ctx.set_table32(True)
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000, precision=GRT_FP32_RELAXED,
                             inner_tol=1e-6)
        say(f"[gpu] star_m1000 relaxed iters={st.iters} fp32={st.fp32_applies} "
            f"resid={st.rel_resid:.2e}")
        _check_solution(ctx, beta, gold, pb, "star_m1000 relaxed")
    finally:
        ctx.close()


def test_curved_m1000():
    """The M=1000 rules between the curved interfaces of the paper's examples 1 and 2:
    K and T on the stored probe, the FP64 and relaxed mixed solutions and their Bragg
    amplitudes against the oracle (tests/golden/curved_m1000_oracle.npz)."""
    from paper_1412_7466_amd.grating import GRT_FP32_RELAXED
    if not os.path.exists(os.path.join(GOLD, "curved_m1000_oracle.npz")):
        pytest.skip("tests/golden/curved_m1000_oracle.npz not generated")
    torch, ctx, gold, pb = _load("curved_m1000")
    try:
        _check_apply(torch, ctx, gold, pb, "curved_m1000")
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
        say(f"[gpu] curved_m1000 FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        _check_solution(ctx, beta, gold, pb, "curved_m1000 FP64")
        ctx.set_table32(True)
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000, precision=GRT_FP32_RELAXED,
                             inner_tol=1e-6)
        say(f"[gpu] curved_m1000 relaxed iters={st.iters} fp32={st.fp32_applies} "
            f"resid={st.rel_resid:.2e}")
        _check_solution(ctx, beta, gold, pb, "curved_m1000 relaxed")
    finally:
        ctx.close()


@pytest.mark.parametrize("inst", [9, 25, 29])
def test_batched_workload_instances(inst):
    """Instances of the batched workload with a stored oracle LU solution
    (tests/golden/batch_oracle.npz): omega = 10, 20 and 40 at P = 10, 15 and 20.  The
    omega = 40 instance checks the high-frequency rules (N, Q, Nw from k3 = 80)."""
    import torch
    from paper_1412_7466_amd.grating import Context
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    gold = np.load(os.path.join(GOLD, "batch_oracle.npz"))
    pb = inputs.batch_problem(inst)
    assert str(gold[f"i{inst}_digest"]) == pb.digest(), "inputs changed: regenerate"
    say(f"[gpu] batch instance {inst}: M={pb.M} P={pb.P} omega={pb.omega}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    beta, st = ctx.solve(tol=1e-12, restart=600, maxit=2000)
    say(f"[gpu] instance {inst}: iters {st.iters} resid {st.rel_resid:.2e}")
    check_orders(beta.cpu().numpy(), gold[f"i{inst}_beta"], gold[f"i{inst}_D"], pb.P, 1e-9,
                 1e-10, tag=f"batch instance {inst} beta")
    og = ctx.bragg(beta)
    p1, p3 = gold[f"i{inst}_prop1"], gold[f"i{inst}_prop3"]
    check_amplitudes(np.concatenate([og["c"][p1], og["d"][p3]]),
                     np.concatenate([gold[f"i{inst}_c"][p1], gold[f"i{inst}_d"][p3]]), 1e-9,
                     tag=f"batch instance {inst} Bragg")
    assert og["flux_err"] < 1e-9
    ctx.close()
