"""grt_eval_field (the total field at arbitrary points) against the oracle's field
(oracle/field.py): every layer, the Rayleigh-Bloch regions above y0 and below -y0,
inside disks and their near copies, and just outside disks.  Points stay more than
six interface-node spacings from the interfaces (where both sides use the node sums
of the discretization).  Bar: 1e-9 of the largest field value sampled."""
import math

import numpy as np
import pytest

from paper_1412_7466_amd import inputs

pytestmark = pytest.mark.gpu


def _points(G, rng):
    pts = []
    gap = 6.5 * G.hs
    for lo, hi in ((G.h + gap, G.y0 + 0.3), (-G.h + gap, G.h - gap), (-G.y0 - 0.3, -G.h - gap)):
        pts.append(np.column_stack([rng.uniform(-0.5 * G.d, 0.5 * G.d, 12), rng.uniform(lo, hi, 12)]))
    for m in range(min(G.M, 5)):
        for l in (0, 1) if m == 0 else (0,):
            for frac in (0.3, 0.95, 1.05, 1.6):
                t = rng.uniform(0, 2 * np.pi)
                pts.append(np.array([[G.cx[m] + l * G.d + frac * G.rad[m] * math.cos(t),
                                      G.cy[m] + frac * G.rad[m] * math.sin(t)]]))
    xy = np.vstack(pts)
    keep = np.abs(np.abs(xy[:, 1]) - G.h) > gap     # not near an interface
    return xy[keep]


@pytest.mark.parametrize("case", ["tiny", "small12", "empty"])
def test_field_matches_oracle(case):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from oracle.field import Field
    from oracle.solver import Reduced
    from paper_1412_7466_amd.grating import Context
    pb = {"tiny": inputs.tiny_m4, "small12": lambda: inputs.small(12, 8, seed=9, phi=0.3),
          "empty": inputs.empty_slab}[case]()
    print(f"[gpu] field case {case} M={pb.M}", flush=True)
    red = Reduced(pb)
    G = red.G
    beta_o = red.solve_lu() if G.M else np.zeros(0)
    F = Field(red, beta_o)
    xy = _points(G, np.random.default_rng(5))
    u_o = F.total(xy[:, 0], xy[:, 1])
    ctx = Context(0)
    ctx.set_problem(pb)
    ctx.build()
    beta = torch.tensor(beta_o, dtype=torch.complex128, device="cuda:0") if G.M else None
    u = ctx.eval_field(beta, xy)
    err = np.abs(u - u_o)
    worst = int(np.argmax(err))
    print(f"[gpu] field {case}: {len(xy)} points, max |u| {np.abs(u_o).max():.3f}, "
          f"max err {err.max():.2e} at {xy[worst]}", flush=True)
    assert err.max() < 1e-9 * np.abs(u_o).max()
    ctx.close()
