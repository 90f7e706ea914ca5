"""The per-voxel relaxation strength map through the HIP path: oracle parity
of heterogeneous 1D/2D/3D cases with smooth random maps in [0.2, 1] (the
kernels of every dimension, the 3D plane kernels included), bit-identity of
an all-ones map with no map, and the map's validation."""
import numpy as np
import pytest

from workloads import configs
from workloads.adapters import oracle_traces, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu


def _case(ndim, shapes, nmech, seed, steps, pml=6):
    c = configs.random_small(ndim, shapes, nmech, 3, seed=seed, steps=steps, pml=pml)
    configs.with_table(c, *configs.random_relaxation_table(seed + 300, c.n_classes, c.nmech))
    return configs.with_strength(c, seed + 500)


@pytest.mark.parametrize("ndim,shapes,nmech,steps", [
    (1, [(400, 1, 1), (257, 1, 1)], 3, 400),
    (2, [(150, 130, 1), (97, 121, 1)], 4, 250),
    (3, [(70, 50, 40), (33, 38, 27)], 4, 120),     # plane kernels (N >= 2)
    (3, [(60, 44, 36)], 1, 120)])                   # marching velocity kernel (N = 1)
def test_strength_map_traces_match_oracle(ndim, shapes, nmech, steps):
    case = _case(ndim, shapes, nmech, 70 + ndim * 10 + nmech, steps)
    print("strength map case", ndim, shapes, nmech, flush=True)
    sim = to_simulation(case)
    sim.step(case.n_steps)
    got = sim.read_receivers()
    ref = oracle_traces(case)
    glob, worst, n = check_traces(got, ref)
    # the map matters: the same case without it differs well above the bar
    plain = configs.Case(**{**case.__dict__, "strength": None})
    ref0 = oracle_traces(plain)
    assert np.linalg.norm(ref0 - ref) / np.linalg.norm(ref) > 1e-3
    report("strength map %dD N=%d shapes=%s: rel_L2 %.3e, worst receiver %.3e (%d reached)"
           % (ndim, nmech, shapes, glob, worst, n))


def test_all_ones_map_is_bitwise_no_map():
    import torch
    case = _case(3, [(70, 50, 40)], 4, 91, 60)
    case.strength = None
    a = to_simulation(case)
    a.step(case.n_steps)
    b = to_simulation(case)
    b.set_strength_map(torch.ones(case.cells(), dtype=torch.float32, device="cuda"))
    b.step(case.n_steps)
    assert np.array_equal(a.read_receivers(), b.read_receivers())


def test_strength_map_validation():
    import torch
    from paper_2606_11103_amd.native import FW_EINVAL, FW_EUNSUPPORTED, FWError
    case = _case(2, [(64, 64, 1)], 2, 92, 20)
    case.nonlinear = False
    sim = to_simulation(case)
    n = case.cells()
    for bad in (1.5, -0.1, float("nan"), float("inf")):
        m = torch.full((n,), 0.5, dtype=torch.float32, device="cuda")
        m[n // 3] = bad
        with pytest.raises(FWError) as ei:
            sim.set_strength_map(m)
        assert ei.value.code == FW_EINVAL
    sim.set_strength_map(torch.full((n,), 0.5, dtype=torch.float32, device="cuda"))
    work = sim.adjoint_workspace(20, 10)
    sim.forward_checkpointed(20, 10, work)
    res = torch.zeros((20, len(case.rec_cell)), dtype=torch.float32, device="cuda")
    with pytest.raises(FWError) as ei:
        sim.adjoint_modulus(20, 10, work, res)
    assert ei.value.code == FW_EUNSUPPORTED
    sim.set_strength_map(None)
    sim.adjoint_modulus(20, 10, work, res)
