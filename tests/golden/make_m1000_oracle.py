"""Write the stored oracle results of the full-size workloads:

  tests/golden/m1000_oracle.npz      M=1000, P=15, omega=20 (the benchmarked workload)
  tests/golden/m1000_p20_oracle.npz  the same geometry at P=20
  tests/golden/star_m1000_oracle.npz the same packing with three-lobed non-circular
                                     inclusions (eq. par1), P=15
  tests/golden/curved_m1000_oracle.npz  the M=1000 rules between the curved interfaces
                                     of the paper's examples 1 and 2, P=15

Each holds the CPU FP64 oracle's GMRES solution to a 1e-12 normalised residual,
its Bragg amplitudes and flux error, the diagonal normalisation D = |H_|n|(k2 r_m)|
and K and T applied to a probe x = D^-1 u, where u has independent standard complex
normal entries in every order (so every order of the output carries weight in the
normalised basis D y).

Calls only oracle/ (and the seeded input generator).  About 10 minutes (P=15) and
20 minutes (P=20) on 8 cores, 3-5 GB of memory: the oracle stores the image-summed
Hankel generator of every (target, source) pair.

    python tests/golden/make_m1000_oracle.py [m1000|m1000_p20|star_m1000|curved_m1000]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1412_7466_amd import inputs  # noqa: E402
from oracle.solver import Reduced  # noqa: E402


def main(case):
    pb = getattr(inputs, case)()
    t0 = time.time()
    red = Reduced(pb, verbose=True)
    t1 = time.time()
    beta = red.solve_gmres(tol=1e-12, maxit=800)
    t2 = time.time()
    out = red.bragg(beta)
    print(f"{case}: setup {t1 - t0:.0f}s  gmres {t2 - t1:.0f}s  iters {red.gmres_iters} "
          f"resid {red.gmres_resid:.2e}  flux {out['flux_err']:.2e}", flush=True)
    rng = np.random.default_rng(123)
    u = rng.standard_normal(red.G.n_beta) + 1j * rng.standard_normal(red.G.n_beta)
    v = u / red.D
    t3 = time.time()
    Kv = red.K_apply(v)
    Tv = red.T_apply(v)
    t4 = time.time()
    np.savez_compressed(os.path.join(ROOT, "tests", "golden", f"{case}_oracle.npz"),
                        digest=pb.digest(), beta=beta, c=out["c"], d=out["d"],
                        orders=out["orders"], prop1=out["prop1"], prop3=out["prop3"],
                        flux_err=out["flux_err"], iters=red.gmres_iters,
                        resid=red.gmres_resid, D=red.D, probe=v, K_probe=Kv, T_probe=Tv,
                        oracle_seconds=np.array([t1 - t0, t2 - t1, (t4 - t3) / 2]))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "m1000")
