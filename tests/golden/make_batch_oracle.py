"""Write tests/golden/batch_oracle.npz: the CPU FP64 oracle's solutions of three
small instances of the batched workload (one per frequency: instances 9, 25 and 29,
M = 203, 241, 272 at omega = 10, 20, 40 with P = 10, 15, 20), solved by LU of the
normalised reduced system, with their Bragg amplitudes and the normalisation D.

Calls only oracle/ (and the seeded input generator).  A few minutes on 8 cores.

    python tests/golden/make_batch_oracle.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1412_7466_amd import inputs  # noqa: E402
from oracle.solver import Reduced  # noqa: E402

INSTANCES = (9, 25, 29)


def main():
    out = {}
    for i in INSTANCES:
        pb = inputs.batch_problem(i)
        t0 = time.time()
        red = Reduced(pb, dense=True)
        beta = red.solve_lu()
        o = red.bragg(beta)
        print(f"instance {i}: M={pb.M} P={pb.P} omega={pb.omega} {time.time() - t0:.0f}s "
              f"flux {o['flux_err']:.2e}", flush=True)
        for k, v in (("digest", pb.digest()), ("beta", beta), ("D", red.D), ("c", o["c"]),
                     ("d", o["d"]), ("prop1", o["prop1"]), ("prop3", o["prop3"]),
                     ("flux_err", o["flux_err"])):
            out[f"i{i}_{k}"] = v
    out["instances"] = np.array(INSTANCES)
    np.savez_compressed(os.path.join(ROOT, "tests", "golden", "batch_oracle.npz"), **out)


if __name__ == "__main__":
    main()
