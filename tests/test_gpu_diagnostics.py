"""FP64 energy and finite-check diagnostics of the HIP path against the
oracle's energy, plus exact-in-FP64 conservation properties on the GPU."""
import numpy as np
import pytest

from workloads import configs
from workloads.adapters import to_oracle, to_simulation

pytestmark = pytest.mark.gpu


def _lossless(ndim, shape, steps, seed):
    c = configs.random_small(ndim, [shape], 1, 3, seed=seed, steps=steps, pml=0, nonlinear=False, noise=0.01,
                             amplitude=1e3)
    C = c.n_classes
    # no relaxation: kappa = 1 and d = 0 make every memory variable vanish
    return configs.with_table(c, np.ones((C, 2)), np.zeros((C, 2, 1)), np.ones((C, 2, 1)))


@pytest.mark.parametrize("ndim,shape", [(2, (96, 80, 1)), (3, (40, 36, 30))])
def test_energy_matches_oracle_and_is_conserved(ndim, shape):
    case = _lossless(ndim, shape, 300, seed=4 + ndim)
    n_src = 60
    case.waves = case.waves.copy()
    case.waves[:, n_src:] = 0.0               # source switched off after 60 steps
    sim = to_simulation(case)
    e_gpu = np.array([sim.energy_step()[0, 0] for _ in range(case.n_steps)])
    orc = to_oracle(case)
    _, e_ref = orc.run(case.n_steps, case.src_cell, case.waves.astype(np.float64)[case.src_wave],
                       case.rec_cell, energy=True)
    rel = np.abs(e_gpu - e_ref) / np.abs(e_ref).max()
    assert rel.max() < 1e-5
    tail = e_gpu[n_src + 1:]
    assert (tail.max() - tail.min()) / tail[0] < 1e-5


def test_energy_steps_equal_plain_steps():
    case = configs.random_small(2, [(80, 70, 1)], 2, 3, seed=3, steps=40)
    configs.with_table(case, *configs.random_relaxation_table(3, case.n_classes, case.nmech))
    a = to_simulation(case)
    a.step(case.n_steps)
    b = to_simulation(case)
    for _ in range(case.n_steps):
        b.energy_step()
    assert np.array_equal(a.read_receivers(), b.read_receivers())


def test_non_finite_pressure_is_reported():
    from paper_2606_11103_amd.native import FWError, FW_ENONFINITE
    case = configs.random_small(2, [(64, 64, 1)], 1, 2, seed=2, steps=20, nonlinear=False)
    configs.with_table(case, *configs.random_relaxation_table(2, case.n_classes, case.nmech))
    case.waves = case.waves.copy()
    case.waves[0, 3] = np.float32(3e38)       # finite input that overflows p to inf
    case.waves[0, 4] = np.float32(3e38)
    sim = to_simulation(case)
    sim.step(4)
    assert sim.first_nonfinite_step() == -1
    with pytest.raises(FWError) as ei:
        for _ in range(3):
            sim.energy_step()
    assert ei.value.code == FW_ENONFINITE
    # the per-step receiver check flags the first trace row with a
    # non-finite value once the overflow has spread to a receiver
    sim.step(case.n_steps - sim.get_step())
    tr = sim.read_receivers()
    bad_rows = np.nonzero(~np.all(np.isfinite(tr), axis=1))[0]
    assert bad_rows.size > 0
    assert sim.first_nonfinite_step() == bad_rows[0]
    sim.reset()
    assert sim.first_nonfinite_step() == -1


def test_loading_a_state_restores_the_non_finite_row():
    """A snapshot carries the first non-finite trace row with the step
    counter: reloading a state saved before the overflow forgets the row
    flagged after it, and stepping on flags it again."""
    case = configs.random_small(2, [(64, 64, 1)], 1, 2, seed=2, steps=20, nonlinear=False)
    configs.with_table(case, *configs.random_relaxation_table(2, case.n_classes, case.nmech))
    case.waves = case.waves.copy()
    case.waves[0, 3] = np.float32(3e38)       # finite input that overflows p to inf
    case.waves[0, 4] = np.float32(3e38)
    sim = to_simulation(case)
    sim.step(2)
    buf = sim.save_state()
    assert sim.first_nonfinite_step() == -1
    sim.step(case.n_steps - 2)
    flagged = sim.first_nonfinite_step()
    assert flagged >= 3
    sim.load_state(buf)
    assert sim.get_step() == 2
    assert sim.first_nonfinite_step() == -1
    sim.step(case.n_steps - 2)
    assert sim.first_nonfinite_step() == flagged
