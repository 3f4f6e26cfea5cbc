"""Full-size parity: the M=1000, P=15 workload the benchmark times, against the
CPU FP64 oracle's stored solution (tests/golden/m1000_oracle.npz, written by
tests/golden/make_m1000_oracle.py from oracle/ only).

Same launch configuration as the benchmark (the work split is a function of M
and the discretization only).  Bars: K applied to a fixed probe vector 1e-9
relative; beta and the propagating Bragg amplitudes 1e-9 relative; flux error
below 1e-9.
"""
import os
import sys

import numpy as np
import pytest

from paper_1412_7466_amd import inputs

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m1000_oracle.npz")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def m1000():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1412_7466_amd.grating import Context
    gold = np.load(GOLD)
    pb = inputs.m1000()
    assert str(gold["digest"]) == pb.digest(), "inputs changed: regenerate the golden file"
    say(f"[gpu] m1000 build M={pb.M} P={pb.P} N={pb.disc.N}")
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    return torch, ctx, gold


def test_m1000_apply(m1000):
    torch, ctx, gold = m1000
    x = torch.tensor(gold["probe"], dtype=torch.complex128, device="cuda:0")
    y = ctx.apply(x).cpu().numpy()
    e = rel(y, gold["K_probe"])
    say(f"[gpu] m1000 K probe rel err {e:.2e}")
    assert e < 1e-9


def _check_solution(ctx, beta, gold, tag):
    b = beta.cpu().numpy()
    e = rel(b, gold["beta"])
    og = ctx.bragg(beta)
    p1, p3 = gold["prop1"], gold["prop3"]
    vg = np.concatenate([og["c"][p1], og["d"][p3]])
    vo = np.concatenate([gold["c"][p1], gold["d"][p3]])
    eb = rel(vg, vo)
    say(f"[gpu] m1000 {tag}: beta rel err {e:.2e}  Bragg rel err {eb:.2e}  "
        f"flux {og['flux_err']:.2e}")
    assert e < 1e-9
    assert eb < 1e-9
    assert og["flux_err"] < 1e-9


def test_m1000_solve_fp64(m1000):
    torch, ctx, gold = m1000
    beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
    say(f"[gpu] m1000 FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
    _check_solution(ctx, beta, gold, "FP64")


def test_m1000_solve_mixed(m1000):
    from paper_1412_7466_amd.grating import GRT_FP32
    torch, ctx, gold = m1000
    beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000, precision=GRT_FP32)
    say(f"[gpu] m1000 mixed iters={st.iters} refine={st.refine_steps} "
        f"resid={st.rel_resid:.2e} {st.seconds:.3f}s")
    _check_solution(ctx, beta, gold, "mixed")


def test_m1000_resident_table(m1000):
    """Same bars with the resident translation table (1 GB at this size)."""
    torch, ctx, gold = m1000
    ctx.set_table(True)
    try:
        x = torch.tensor(gold["probe"], dtype=torch.complex128, device="cuda:0")
        e = rel(ctx.apply(x).cpu().numpy(), gold["K_probe"])
        say(f"[gpu] m1000 table: K probe rel err {e:.2e}")
        assert e < 1e-9
        beta, st = ctx.solve(tol=1e-12, restart=200, maxit=1000)
        say(f"[gpu] m1000 table FP64 iters={st.iters} resid={st.rel_resid:.2e} {st.seconds:.3f}s")
        _check_solution(ctx, beta, gold, "FP64 table")
    finally:
        ctx.set_table(False)
