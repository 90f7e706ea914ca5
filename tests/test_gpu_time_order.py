"""The time-space-domain staggered coefficients (fw_set_time_space_stencil,
the fourth-order-in-time operator of Sec. 3.3) on the GPU against the FP64
oracle run with the same set: 1D (resident step), 2D tile kernels, 3D plane
kernels and the adjoint.  The kernels are those of the Taylor set; only the
coefficient values differ, so the bar is the same (global and worst reached
receiver <= 1e-4), and the runs must differ from the Taylor-set runs by far
more than that."""
import dataclasses

import numpy as np
import pytest

from workloads import configs
from workloads.adapters import oracle_traces, to_oracle, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu


def _with_ts(case):
    return dataclasses.replace(case, fd_c_ref=float(np.mean(case.c)))


def _cases(name):
    if name == "1d_ragged_resident":
        c = configs.random_small(1, [(8192, 1, 1), (3001, 1, 1), (77, 1, 1)], 2, 3, seed=70, steps=1500)
    elif name == "2d_tile":
        c = configs.random_small(2, [(150, 130, 1)], 4, 3, seed=71, steps=300)
    elif name == "3d_plane":
        c = configs.random_small(3, [(70, 50, 40)], 4, 3, seed=72, steps=150)
    elif name == "3d_N2_ragged":
        c = configs.random_small(3, [(67, 37, 29), (40, 33, 30)], 2, 3, seed=73, steps=120, pml=5)
    else:
        raise KeyError(name)
    return configs.with_table(c, *configs.random_relaxation_table(170 + len(name), c.n_classes, c.nmech))


@pytest.mark.parametrize("name", ["1d_ragged_resident", "2d_tile", "3d_plane", "3d_N2_ragged"])
def test_time_space_set_matches_oracle(name):
    base = _cases(name)
    case = _with_ts(base)
    print("time-space case", name, case.shapes, "N=%d" % case.nmech, "c_ref=%.1f" % case.fd_c_ref, flush=True)
    sim = to_simulation(case)
    from oracle import fdcoef
    ref_coef = fdcoef.time_space_coefficients(case.fd_c_ref * case.dt / case.dx, 4)
    coef, b = sim.stencil()
    assert np.max(np.abs(np.array(coef) - ref_coef) / np.abs(ref_coef)) < 1e-13 and b == 0.0
    sim.step(case.n_steps)
    got = sim.read_receivers()
    del sim
    ref = oracle_traces(case)
    glob, worst, n = check_traces(got, ref)
    # the option is in effect: the Taylor-set oracle run is far from both
    ref_taylor = oracle_traces(base)
    sep = float(np.linalg.norm(ref_taylor - ref) / np.linalg.norm(ref))
    report("time-space stencil %s rel_L2=%.3e worst_receiver=%.3e (%d reached); Taylor-set run differs by %.3e"
           % (name, glob, worst, n, sep))
    assert sep > 100 * max(glob, 1e-6)


def test_time_space_set_adjoint_matches_fp64_adjoint():
    import torch
    from oracle.solver import misfit_gradient
    c = configs.random_small(2, [(64, 64, 1), (48, 72, 1)], 4, 3, seed=74, steps=160, pml=8,
                             nonlinear=False, noise=0.01, n_rec=16)
    case = _with_ts(configs.with_table(c, *configs.random_relaxation_table(174, c.n_classes, c.nmech)))
    obs = np.zeros((case.n_steps, len(case.rec_cell)))
    sim = to_simulation(case)
    n, ckpt = case.n_steps, 23
    work = sim.adjoint_workspace(n, ckpt)
    sim.forward_checkpointed(n, ckpt, work)
    tr = sim.read_receivers_device()
    res = (case.dt * (tr.double() - torch.as_tensor(obs, device=tr.device))).float()
    gK, gs = sim.adjoint_modulus(n, ckpt, work, res)
    gK, gs = gK.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
    oK, os_ = [], []
    for d in range(len(case.shapes)):
        osim = to_oracle(case, d)
        sm = case.src_domain == d
        rm = np.nonzero(case.rec_domain == d)[0]
        waves = case.waves.astype(np.float64)[case.src_wave[sm]]
        _, k, s, _ = misfit_gradient(osim, n, case.src_cell[sm], waves, case.rec_cell[rm], obs[:, rm])
        oK.append(k)
        os_.append(s)
    oK, os_ = np.concatenate(oK), np.concatenate(os_)
    rK = float(np.linalg.norm(gK - oK) / np.linalg.norm(oK))
    rs = float(np.linalg.norm(gs - os_) / np.linalg.norm(os_))
    report("time-space stencil adjoint 2D N=4 rel_L2 gK=%.3e gs=%.3e" % (rK, rs))
    assert np.abs(oK).max() > 0 and np.abs(os_).max() > 0
    assert rK <= 1e-4 and rs <= 1e-4


def _widened(case):
    return dataclasses.replace(case, fd_c_ref=float(np.mean(case.c)), fd_widened=True)


def _run(case, opts=None, steps=None):
    sim = to_simulation(case)
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    sim.step(case.n_steps if steps is None else steps)
    tr = sim.read_receivers()
    del sim
    return tr


@pytest.mark.parametrize("nmech", [1, 4])
def test_widened_stencil_2d_tiles_match_oracle(nmech):
    """The widened 2D stencil (fourth order in time in every direction) on the
    2D tile kernels with 4-, 8- and 16-row tiles, over a ragged batch of five
    domains (partial tiles on both axes, CPML, noise, nonlinearity), against
    the FP64 oracle with the same stencil; with a strength map too (N = 4)."""
    from paper_2606_11103_amd.native import FW_OPT_PLANE_ROWS
    from oracle import fdcoef
    shapes = [(70, 21, 1), (33, 38, 1), (130, 97, 1), (64, 61, 1), (65, 19, 1)]
    c = configs.random_small(2, shapes, nmech, 3, seed=80 + nmech, steps=200, pml=5)
    base = configs.with_table(c, *configs.random_relaxation_table(180 + nmech, c.n_classes, c.nmech))
    case = _widened(base)
    print("widened stencil, ragged 2D batch, N=%d" % nmech, flush=True)
    sim = to_simulation(case)
    coef, b = sim.stencil()
    rc, rb = fdcoef.isotropic_time_space_coefficients(case.fd_c_ref * case.dt / case.dx, 2, 4)
    assert np.max(np.abs(np.array(coef) - rc) / np.abs(rc)) < 1e-13 and abs(b - rb) <= 1e-15 * rb
    del sim
    runs = {rows: _run(case, {FW_OPT_PLANE_ROWS: rows}) for rows in (4, 8, 16)}
    assert np.array_equal(runs[4], runs[8]) and np.array_equal(runs[4], runs[16])
    ref = oracle_traces(case)
    glob, worst, n = check_traces(runs[8], ref)
    sep = float(np.linalg.norm(oracle_traces(_with_ts(base)) - ref) / np.linalg.norm(ref))
    report("widened stencil 2D ragged batch N=%d: rel_L2=%.3e worst_receiver=%.3e (%d reached); on-axis set "
           "differs by %.3e" % (nmech, glob, worst, n, sep))
    assert sep > 100 * max(glob, 1e-6)
    if nmech == 4:
        smap = configs.with_strength(case, 9, 0.2, 1.0)
        got = _run(smap, {FW_OPT_PLANE_ROWS: 8})
        glob_s, worst_s, n_s = check_traces(got, oracle_traces(smap))
        report("widened stencil 2D ragged batch N=4 with a strength map: rel_L2=%.3e worst_receiver=%.3e"
               % (glob_s, worst_s))


def test_widened_stencil_rejects_paths_without_it():
    """Marching 2D kernels and the adjoint do not implement the widened
    stencil: stepping on them and the adjoint fail with FW_EUNSUPPORTED
    instead of running another scheme; restoring the Taylor set lifts it."""
    import torch
    from paper_2606_11103_amd.native import FW_EUNSUPPORTED, FW_OPT_PLANE_KERNELS, FWError
    c = configs.random_small(2, [(64, 64, 1)], 2, 3, seed=86, steps=40, pml=6, nonlinear=False)
    case = _widened(configs.with_table(c, *configs.random_relaxation_table(186, c.n_classes, c.nmech)))
    sim = to_simulation(case)
    sim.set_option(FW_OPT_PLANE_KERNELS, 0)
    with pytest.raises(FWError) as e:
        sim.step(1)
    assert e.value.code == FW_EUNSUPPORTED
    sim.set_option(FW_OPT_PLANE_KERNELS, 1)
    work = sim.adjoint_workspace(case.n_steps, 10)
    sim.forward_checkpointed(case.n_steps, 10, work)        # a forward run on the tile kernels
    res = torch.zeros((case.n_steps, len(case.rec_cell)), dtype=torch.float32, device=sim.device)
    with pytest.raises(FWError) as e:
        sim.adjoint_modulus(case.n_steps, 10, work, res)
    assert e.value.code == FW_EUNSUPPORTED
    sim.set_widened_stencil(0.0)
    sim.set_option(FW_OPT_PLANE_KERNELS, 0)
    sim.reset()
    sim.step(5)


def test_widened_stencil_long_horizon_512():
    """The widened 2D stencil over 2000 steps on 512 x 512 cells (N = 4, 24-cell
    CPML, noise, nonlinear, 24 receivers) against the live FP64 oracle: the
    global and the worst reached receiver's relative L2 within the bar."""
    c = configs.random_small(2, [(512, 512, 1)], 4, 3, seed=88, steps=2000, pml=24, n_rec=24)
    case = _widened(configs.with_table(c, *configs.random_relaxation_table(188, c.n_classes, c.nmech)))
    print("widened stencil, 512^2, 2000 steps", flush=True)
    got = _run(case)
    ref = oracle_traces(case)
    glob, worst, n = check_traces(got, ref)
    report("widened stencil 2D 512x512 N=4, 2000 steps: rel_L2=%.3e worst_receiver=%.3e (%d of %d reached)"
           % (glob, worst, n, len(case.rec_cell)))


def test_widened_stencil_graph_eager_resume_and_switch_are_bitwise():
    """With the widened stencil: eager launches, graph replays of 16 and 7
    steps, and a save / advance / reload / resume give the same bits; setting
    the stencil drops the captured graph, so switching back to the Taylor set
    mid-life reproduces a plain Taylor run from a reset."""
    from paper_2606_11103_amd.native import FW_OPT_GRAPH_STEPS
    c = configs.random_small(2, [(150, 130, 1), (77, 96, 1)], 4, 3, seed=89, steps=240, pml=6)
    base = configs.with_table(c, *configs.random_relaxation_table(189, c.n_classes, c.nmech))
    case = _widened(base)
    a = _run(case, {FW_OPT_GRAPH_STEPS: 0})
    assert np.array_equal(a, _run(case, {FW_OPT_GRAPH_STEPS: 16}))
    assert np.array_equal(a, _run(case, {FW_OPT_GRAPH_STEPS: 7}))
    n = case.n_steps
    sim = to_simulation(case)
    sim.step(n // 2)
    buf = sim.save_state()
    sim.step(17)
    sim.load_state(buf)
    sim.step(n - n // 2)
    assert np.array_equal(sim.read_receivers(), a)
    # back to the Taylor set on the same Simulation (the widened graph is dropped)
    sim.set_widened_stencil(0.0)
    sim.reset()
    sim.step(n)
    assert np.array_equal(sim.read_receivers(), _run(base))
    assert not np.array_equal(a, _run(base))
