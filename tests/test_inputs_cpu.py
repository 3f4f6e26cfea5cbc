"""The seeded workload generators (paper_1412_7466_amd/inputs.py) on the CPU: the
packing rules they promise, determinism, and the distributions of the batched
mixed-precision workload and the warm-start sets."""
import math

import numpy as np

from paper_1412_7466_amd import inputs


def _packing_ok(pb, gap, clearance):
    """disks inside the cell and the middle layer with the clearance, pairwise gaps
    (minimum image in x) at least gap"""
    assert np.all(np.abs(pb.x) <= pb.d / 2)
    assert np.all(np.abs(pb.y) + pb.radius <= pb.h - clearance + 1e-12)
    assert inputs.min_image_gap(pb.x, pb.y, pb.radius, pb.d) >= gap - 1e-12


def test_m1000_rules():
    pb = inputs.m1000()
    assert pb.M == 1000 and pb.P == 15 and pb.omega == 20.0
    assert abs(pb.phi + math.pi / 5) < 1e-15
    assert np.all((pb.radius >= 0.004) & (pb.radius <= 0.012))
    assert np.all((pb.n_incl >= 1.5) & (pb.n_incl <= 3.0))
    _packing_ok(pb, 0.002, 0.02)


def test_batch_problem_distribution_and_determinism():
    cells = [(0, 0), (1, 5), (2, 10), (0, 15), (1, 12), (2, 3)]
    pbs = [inputs.batch_problem(i, cells) for i in range(12)]
    for i, pb in enumerate(pbs):
        assert 200 <= pb.M <= 4000
        wi, ai = cells[i % len(cells)]
        assert pb.P == inputs.BATCH_PS[wi]          # P goes with omega
        assert pb.seed == 3000 + i
        assert pb.omega == inputs.BATCH_OMEGAS[wi]
        assert pb.phi == inputs.BATCH_PHIS[ai]
        assert abs(pb.phi) <= math.pi / 3 + 1e-15
    # small instances are checked for the packing rules in full (large ones take
    # seconds of pure-Python checking)
    for pb in pbs:
        if pb.M <= 600:
            _packing_ok(pb, 0.002, 0.02)
    again = inputs.batch_problem(3, cells)
    assert again.M == pbs[3].M and np.array_equal(again.x, pbs[3].x)
    # the default grid covers 3 frequencies x 16 angles, angles equally spaced
    ph = np.array(inputs.BATCH_PHIS)
    assert len(ph) == 16 and np.allclose(np.diff(ph), ph[1] - ph[0])
    assert abs(ph[0] + math.pi / 3) < 1e-15 and abs(ph[-1] - math.pi / 3) < 1e-12
    full = [inputs.batch_problem(i) for i in range(3)]
    assert [p.omega for p in full] == [10.0, 20.0, 40.0]
    assert [p.P for p in full] == [10, 15, 20]
    assert inputs.batch_problem(3).phi == inputs.BATCH_PHIS[1]


def test_problems_of_one_cell_share_the_discretization():
    a = inputs.warm_problem(0, held_out=True, M_range=(200, 300))
    b = inputs.warm_problem(len(inputs.WARM_OMEGAS) * len(inputs.WARM_PHIS),
                            held_out=True, M_range=(200, 300))
    assert (a.omega, a.phi) == (b.omega, b.phi)
    assert a.disc == b.disc
