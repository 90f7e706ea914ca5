"""Label-wise inversion through the HIP adjoint: the sound speed (and the
attenuation) of a two-label 2D medium recovered from synthetic traces of the
true medium."""
import numpy as np
import pytest

from workloads import configs
from reporting import report

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_2606_11103_amd.autograd import Problem, simulate
    case = configs.random_small(2, [(80, 80, 1)], 2, 2, seed=31, steps=220, pml=8, nonlinear=False, noise=0.0,
                                n_rec=24)
    case = configs.with_table(case, *configs.random_relaxation_table(131, case.n_classes, case.nmech))
    lab = case.class_maps[0]
    prob = Problem(ndim=2, shapes=case.shapes, dx=case.dx, dt=case.dt, nmech=case.nmech, pml_cells=case.pml_cells,
                   labels=[lab], rho=case.rho, alpha0_ref=case.alpha0, kappa=case.kappa, d=case.d,
                   alpha=case.alpha, src_domain=case.src_domain, src_cell=case.src_cell, src_wave=case.src_wave,
                   waves=case.waves, rec_domain=case.rec_domain, rec_cell=case.rec_cell, n_steps=case.n_steps,
                   ckpt_every=40, pml_params=(1e-4, 1e6, float(case.c.max()) * 1.05))
    flat = lab.reshape(-1).astype(np.int64)
    with torch.no_grad():
        obs = simulate(torch.tensor(case.c[flat]), torch.tensor(case.alpha0[flat]), prob).double()
    return case, prob, obs


def test_sound_speed_of_two_labels_is_recovered():
    from paper_2606_11103_amd.inversion import invert_labels
    case, prob, obs = _setup()
    c0 = case.c * np.array([1.015, 0.985])
    res = invert_labels(prob, obs, c0, case.alpha0, iters=6, step_c=10.0)
    err0, err = np.abs(c0 - case.c).max(), np.abs(res.c - case.c).max()
    report("inversion c: misfit %.3e -> %.3e in %d steps; max |c - c_true| %.2f -> %.4f m/s"
           % (res.misfits[0], res.misfits[-1], len(res.steps), err0, err))
    assert all(b < a for a, b in zip(res.misfits, res.misfits[1:]))
    assert res.misfits[-1] < 1e-3 * res.misfits[0]
    assert err < 0.05 * err0


def test_speed_and_attenuation_of_two_labels_are_recovered():
    from paper_2606_11103_amd.inversion import invert_labels
    case, prob, obs = _setup()
    c0 = case.c * np.array([1.01, 0.99])
    a0 = case.alpha0 * np.array([1.25, 0.75])
    res = invert_labels(prob, obs, c0, a0, iters=30, invert_alpha=True, step_c=6.0, step_a=0.3)
    ec0, ec = np.abs(c0 - case.c).max(), np.abs(res.c - case.c).max()
    ea0, ea = np.abs(a0 / case.alpha0 - 1).max(), np.abs(res.alpha0 / case.alpha0 - 1).max()
    report("inversion c+alpha0: misfit %.3e -> %.3e in %d steps; max |c - c_true| %.2f -> %.4f m/s; "
           "max rel alpha0 error %.3f -> %.4f" % (res.misfits[0], res.misfits[-1], len(res.steps), ec0, ec, ea0, ea))
    assert all(b < a for a, b in zip(res.misfits, res.misfits[1:]))
    assert res.misfits[-1] < 1e-6 * res.misfits[0]
    assert ec < 1e-2 * ec0 and ea < 1e-2 * ea0
