"""The allocation-free energy step against the allocating one, through the
C ABI: identical outputs and traces on two calls in a row, the second on a
smaller input (the calls share the library's fixed scratch), plus its size
and call-order errors."""
import numpy as np
import pytest

from workloads import configs
from workloads.adapters import to_simulation

pytestmark = pytest.mark.gpu


def _case(shapes, ndim, seed, nmech=2, steps=12):
    c = configs.random_small(ndim, shapes, nmech, 3, seed=seed, steps=steps, pml=6, nonlinear=True, noise=0.01)
    return configs.with_table(c, *configs.random_relaxation_table(seed + 7, c.n_classes, c.nmech))


def _compare(case, k):
    ref = to_simulation(case)
    new = to_simulation(case)
    ref.step(1)
    new.step(1)
    for _ in range(k):
        e_ref = ref.energy_step()
        e_new = new.energy_step_noalloc()
        assert np.array_equal(e_ref, e_new), (e_ref, e_new)
    assert np.abs(e_ref[:, 0]).max() > 0
    assert np.array_equal(ref.read_receivers(), new.read_receivers())
    return e_new


def test_noalloc_energy_step_matches_the_allocating_one():
    from paper_2606_11103_amd.native import FW_EINVAL, FW_ESTATE, FWError
    big = _case([(180, 150, 1), (96, 130, 1)], 2, seed=31)
    small = _case([(40, 36, 30)], 3, seed=32)
    _compare(big, 6)
    _compare(small, 6)       # second call, smaller input, same scratch
    # the tile lists must exist (building them allocates)
    fresh = to_simulation(small)
    with pytest.raises(FWError) as ei:
        fresh.energy_step_noalloc()
    assert ei.value.code == FW_ESTATE
    # beyond the scratch size (8 Mi cells): rejected with a clear error
    huge = _case([(2060, 4100, 1)], 2, seed=33, nmech=1, steps=2)
    sim = to_simulation(huge)
    sim.step(1)
    with pytest.raises(FWError) as ei:
        sim.energy_step_noalloc()
    assert ei.value.code == FW_EINVAL and "allocation-free limit" in str(ei.value)
