"""Write the FP64 oracle's receiver traces for the full 2D two-layer workload.

2048 x 2048 cells, dx = 0.03 mm, N = 4, 24-cell CPML, nonlinear (B/A 6 and 9),
plane-wave line source, 128 receivers, 4000 steps (1.68e10 cell-updates:
about 10-30 minutes of host time with OpenMP).  The relaxation tables are the
cached host fits of the two classes, step-matched to the run's time step; they
are stored beside the traces so that the GPU test feeds the library exactly
the inputs the oracle was given.  The
traces are stored rounded to FP32 (relative error 6e-8, far below the 1e-4
parity bound).

Only the oracle computes here (the seeded workload module only builds the
inputs).  Run from the repository root:
    python tests/golden/make_two_layer_traces.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "two_layer_2d_2048_oracle.npz")


def main(steps=4000):
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from oracle import solver
    from paper_2606_11103_amd import relax
    from workloads import configs
    from workloads.adapters import oracle_traces
    solver.build()
    case = configs.two_layer_2d(steps=steps)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    t0 = time.time()
    tr = oracle_traces(case, steps)
    dt = time.time() - t0
    np.savez_compressed(OUT, traces=tr.astype(np.float32), kappa=kappa, d=d, alpha=al, steps=steps,
                        c=case.c, rho=case.rho, dx=case.dx, dt=case.dt, rec_cell=case.rec_cell,
                        src_cell=case.src_cell, wave=case.waves[0])
    print("wrote %s: %d steps x %d receivers in %.0f s" % (OUT, tr.shape[0], tr.shape[1], dt))


if __name__ == "__main__":
    main()
