"""Write the FP64 oracle's receiver traces for a 256 x 256 x 192 instance of
the 3D heterogeneous workload over its full 2000 steps.

The instance is the benchmark recipe at the size of the centre crop the
oracle can hold: 8 tissue classes (seed 3) on a smoothed label field, +-1 %
per-voxel speed perturbation (seed 33), nonlinear (B/A 5-10), N = 4, 24-cell
CPML, dt at CFL 0.4 on 1650 * 1.01 m/s, the focused 64-element array
(2.5 MHz, 0.5 MPa) and its receivers (element centres and on-axis points).
The relaxation tables are the cached host fits of the 8 classes, step-matched
to the run's time step; they are stored beside the traces so that the GPU
test feeds the library exactly the inputs the oracle was given.  Traces are
stored rounded to FP32 (relative error 6e-8, far below the 1e-4 bound).
2.5e10 cell-updates: about 10 minutes of host time with OpenMP.

Only the oracle computes here (the seeded workload module only builds the
inputs).  Run from the repository root:
    python tests/golden/make_3d_instance_traces.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "heterogeneous_3d_256x256x192_oracle.npz")
SHAPE = (256, 256, 192)


def main(steps=2000):
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from oracle import solver
    from paper_2606_11103_amd import relax
    from workloads import configs
    from workloads.adapters import oracle_traces
    solver.build()
    case = configs.heterogeneous_3d(shape=SHAPE, steps=steps)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    t0 = time.time()
    tr = oracle_traces(case, steps)
    dt = time.time() - t0
    np.savez_compressed(OUT, traces=tr.astype(np.float32), kappa=kappa, d=d, alpha=al, steps=steps,
                        c=case.c, rho=case.rho, dx=case.dx, dt=case.dt, rec_cell=case.rec_cell,
                        src_cell=case.src_cell, waves=case.waves)
    print("wrote %s: %d steps x %d receivers in %.0f s" % (OUT, tr.shape[0], tr.shape[1], dt))


if __name__ == "__main__":
    main()
