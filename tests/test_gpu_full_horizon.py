"""Every workload at its full step count against the FP64 oracle, with the
global and the worst-reached-receiver relative L2 error of the receiver
traces (both <= 1e-4), in the launch configuration the benchmark uses.

* 3D heterogeneous recipe (8 calibrated step-matched classes, focused array,
  +-1 % speed perturbation, nonlinear, N = 4, 24-cell CPML, 2000 steps) on a
  128 x 128 x 96 instance (oracle live, about 30 s on 16 host cores), the
  same with N = 2, and on a 256 x 256 x 192 instance (oracle traces stored
  by tests/golden/make_3d_instance_traces.py);
* the 64-shot batched 2D launch over all 3000 steps: the smallest, the
  largest and two middle shots against the oracle;
* the 544-domain 1D sweep over its full 14 800 steps: eight domains spanning
  the (alpha0, y) grid against the oracle;
* the adjoint workload's forward run (16 shots of 1024^2, 3000 steps): two
  shots against the oracle.
The 2D homogeneous (600 steps) and two-layer (4000 steps) workloads run in
test_gpu_parity.py and test_gpu_fullsize.py with the same two figures."""
import os

import numpy as np
import pytest

from workloads import configs
from workloads.adapters import to_oracle, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_3D = os.path.join(HERE, "golden", "heterogeneous_3d_256x256x192_oracle.npz")


def _calibrated(case):
    from paper_2606_11103_amd import relax
    k, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech, allow_fit=False,
                                   dt=case.dt)
    return configs.with_table(case, k, d, al)


def _oracle_domain(case, dom):
    """FP64 traces of one domain: [steps][receivers of that domain]."""
    sim = to_oracle(case, dom)
    sm = case.src_domain == dom
    rm = np.nonzero(case.rec_domain == dom)[0]
    waves = case.waves.astype(np.float64)[case.src_wave[sm]]
    rec, _ = sim.run(case.n_steps, case.src_cell[sm], waves, case.rec_cell[rm])
    return rm, rec


def _gpu(case):
    sim = to_simulation(case)
    sim.step(case.n_steps)
    tr = sim.read_receivers().astype(np.float64)
    del sim
    return tr


def test_3d_recipe_128x128x96_all_2000_steps():
    case = _calibrated(configs.heterogeneous_3d(shape=(128, 128, 96), steps=2000, n_elem=16))
    print("3D instance", case.shapes, "steps", case.n_steps, flush=True)
    got = _gpu(case)
    _, ref = _oracle_domain(case, 0)
    glob, worst, n = check_traces(got, ref)
    report("full horizon: 3D heterogeneous 128x128x96 N=4 nonlinear noise, 2000 steps: rel_L2 %.3e, worst receiver "
           "%.3e (%d of %d reached), peak %.3g Pa" % (glob, worst, n, ref.shape[1], np.abs(ref).max()))


def test_3d_recipe_at_the_papers_n2_128x128x96_all_2000_steps():
    """The 3D recipe with N = 2 (the paper's mechanism count and the library's
    N <= 2 launch shape: 8-row plane tiles, two planes per velocity tile)."""
    case = _calibrated(configs.heterogeneous_3d(shape=(128, 128, 96), steps=2000, n_elem=16, nmech=2))
    print("3D instance N=2", case.shapes, "steps", case.n_steps, flush=True)
    got = _gpu(case)
    _, ref = _oracle_domain(case, 0)
    glob, worst, n = check_traces(got, ref)
    report("full horizon: 3D heterogeneous 128x128x96 N=2 nonlinear noise, 2000 steps: rel_L2 %.3e, worst receiver "
           "%.3e (%d of %d reached), peak %.3g Pa" % (glob, worst, n, ref.shape[1], np.abs(ref).max()))


def test_3d_recipe_256x256x192_all_2000_steps_against_stored_oracle():
    g = np.load(GOLDEN_3D)
    steps = int(g["steps"])
    case = configs.heterogeneous_3d(shape=(256, 256, 192), steps=steps)
    np.testing.assert_array_equal(g["c"], case.c)
    np.testing.assert_array_equal(g["rho"], case.rho)
    np.testing.assert_array_equal(g["rec_cell"], case.rec_cell)
    np.testing.assert_array_equal(g["src_cell"], case.src_cell)
    np.testing.assert_array_equal(g["waves"], case.waves)
    assert float(g["dx"]) == case.dx and float(g["dt"]) == case.dt
    configs.with_table(case, g["kappa"], g["d"], g["alpha"])
    print("3D instance", case.shapes, "steps", steps, flush=True)
    got = _gpu(case)
    ref = g["traces"].astype(np.float64)
    glob, worst, n = check_traces(got, ref)
    report("full horizon: 3D heterogeneous 256x256x192 N=4 nonlinear noise, 2000 steps: rel_L2 %.3e, worst receiver "
           "%.3e (%d of %d reached), peak %.3g Pa" % (glob, worst, n, ref.shape[1], np.abs(ref).max()))


def test_batched_64_shots_all_3000_steps():
    case = configs.batched_2d()
    configs.with_table(case, *configs.random_relaxation_table(4000, case.n_classes, case.nmech))
    print("64-shot batch", case.cells(), "cells, steps", case.n_steps, flush=True)
    got = _gpu(case)
    sides = np.array([s[0] for s in case.shapes])
    order = np.argsort(sides)
    picks = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), int(order[-1])]
    for dom in picks:
        print("oracle shot", dom, case.shapes[dom], flush=True)
        rm, ref = _oracle_domain(case, dom)
        glob, worst, n = check_traces(got[:, rm], ref)
        report("full horizon: batched 2D shot %d (%dx%d) of 64, 3000 steps: rel_L2 %.3e, worst receiver %.3e "
               "(%d of %d reached)" % (dom, sides[dom], sides[dom], glob, worst, n, len(rm)))


def test_sweep_544_domains_full_length():
    case = _calibrated(configs.sweep_1d())
    print("1D sweep", len(case.shapes), "domains, steps", case.n_steps, flush=True)
    got = _gpu(case)
    nd = len(case.shapes)
    # corners and middle of the (alpha0, y) grid: 32 alpha0 x 17 y, y fastest
    picks = [0, 16, 8 * 17 + 5, 15 * 17 + 8, 16 * 17 + 11, 24 * 17 + 3, 31 * 17, nd - 1]
    for dom in picks:
        rm, ref = _oracle_domain(case, dom)
        glob, worst, n = check_traces(got[:, rm], ref)
        report("full horizon: 1D sweep domain %d (alpha0 %.4g, y %.2f), %d steps: rel_L2 %.3e, worst receiver %.3e "
               "(%d of %d reached)" % (dom, case.alpha0[dom], case.y[dom], case.n_steps, glob, worst, n, len(rm)))


def test_adjoint_workload_forward_all_3000_steps():
    case = _calibrated(configs.adjoint_2d())
    print("adjoint workload", len(case.shapes), "shots, steps", case.n_steps, flush=True)
    got = _gpu(case)
    for dom in (0, len(case.shapes) - 1):
        rm, ref = _oracle_domain(case, dom)
        glob, worst, n = check_traces(got[:, rm], ref)
        report("full horizon: adjoint workload shot %d (1024x1024, N=4), 3000 steps: rel_L2 %.3e, worst receiver "
               "%.3e (%d of %d reached)" % (dom, glob, worst, n, len(rm)))
