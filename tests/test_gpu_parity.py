"""HIP path vs the FP64 oracle, element by element on the receiver traces
(relative L2 over [steps x receivers], FP64 sums, bar 1e-4), plus the
bitwise invariances of the HIP path itself (launch path, tiling, batching,
resume)."""
import time
import zlib

import numpy as np
import pytest

from workloads import configs
from workloads.adapters import oracle_traces, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(name):
    if name == "2d_homogeneous_256":
        # the full 2D homogeneous workload with its calibrated, step-matched table
        from paper_2606_11103_amd import relax
        c = configs.homogeneous_2d(256, 600)
        k, d, al, _ = relax.tables_for(dict(c=c.c, alpha0=c.alpha0, y=c.y), c.nmech, allow_fit=False, dt=c.dt)
        return configs.with_table(c, k, d, al)
    elif name == "2d_random_N4":
        c = configs.random_small(2, [(150, 130, 1)], 4, 3, seed=1, steps=300)
    elif name == "2d_random_N1_linear":
        c = configs.random_small(2, [(131, 97, 1)], 1, 2, seed=6, steps=250, nonlinear=False, noise=0.0)
    elif name == "3d_random_N4":
        c = configs.random_small(3, [(70, 50, 40)], 4, 3, seed=2, steps=150)
    elif name == "3d_random_N2_ragged":
        c = configs.random_small(3, [(67, 37, 29)], 2, 4, seed=8, steps=120, pml=5)
    elif name == "3d_random_N3":
        c = configs.random_small(3, [(40, 33, 30)], 3, 2, seed=9, steps=100, pml=4)
    elif name == "1d_batched_N2":
        c = configs.random_small(1, [(300, 1, 1), (257, 1, 1), (129, 1, 1)], 2, 2, seed=3, steps=400)
    elif name == "2d_batched_N3":
        c = configs.random_small(2, [(100, 90, 1), (77, 130, 1), (65, 65, 1)], 3, 2, seed=4, steps=200)
    elif name == "1d_batched_N4":
        c = configs.random_small(1, [(512, 1, 1), (203, 1, 1), (77, 1, 1)], 4, 3, seed=10, steps=500)
    elif name == "1d_N1_linear":
        c = configs.random_small(1, [(333, 1, 1)], 1, 2, seed=11, steps=400, nonlinear=False, noise=0.0)
    elif name == "3d_closed_N2":
        c = configs.random_small(3, [(45, 38, 33)], 2, 3, seed=12, steps=90, pml=0)
    else:
        raise KeyError(name)
    return configs.with_table(c, *configs.random_relaxation_table(zlib.crc32(name.encode()) % 1000, c.n_classes, c.nmech))


PARITY_CASES = ["2d_homogeneous_256", "2d_random_N4", "2d_random_N1_linear", "3d_random_N4",
                "3d_random_N2_ragged", "3d_random_N3", "1d_batched_N2", "2d_batched_N3",
                "1d_batched_N4", "1d_N1_linear", "3d_closed_N2"]


@pytest.mark.parametrize("name", PARITY_CASES)
def test_traces_match_oracle(name):
    case = _case(name)
    print("case", name, case.shapes, "N=%d" % case.nmech, "steps=%d" % case.n_steps, flush=True)
    sim = to_simulation(case)
    sim.step(case.n_steps)
    got = sim.read_receivers()
    ref = oracle_traces(case)
    glob, worst, n = check_traces(got, ref)
    report("%s rel_L2=%.3e worst_receiver=%.3e (%d of %d reached) steps=%d"
           % (name, glob, worst, n, len(case.rec_cell), case.n_steps))


def _run(case, steps=None, opts=None):
    sim = to_simulation(case)
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    sim.step(case.n_steps if steps is None else steps)
    return sim, sim.read_receivers()


def test_graph_and_eager_paths_are_bitwise_identical():
    from paper_2606_11103_amd.native import FW_OPT_GRAPH_STEPS
    case = _case("3d_random_N4")
    _, a = _run(case, opts={FW_OPT_GRAPH_STEPS: 0})
    _, b = _run(case, opts={FW_OPT_GRAPH_STEPS: 16})
    _, c = _run(case, opts={FW_OPT_GRAPH_STEPS: 7})
    assert np.array_equal(a, b) and np.array_equal(a, c)
    # fw_prepare captures the graph ahead (twice: the second call finds it
    # current) and leaves the state alone; an option change after it rebuilds
    sim = to_simulation(case)
    sim.prepare()
    sim.prepare()
    assert sim.get_step() == 0
    sim.step(case.n_steps)
    assert np.array_equal(a, sim.read_receivers())
    sim = to_simulation(case)
    sim.prepare()
    sim.set_option(FW_OPT_GRAPH_STEPS, 5)
    sim.prepare()
    sim.step(case.n_steps)
    assert np.array_equal(a, sim.read_receivers())


def test_tiling_does_not_change_results():
    from paper_2606_11103_amd.native import (FW_OPT_MARCH_CHUNK, FW_OPT_PERSISTENT, FW_OPT_PLANE_KERNELS,
                                             FW_OPT_ROWS_PER_THREAD, FW_OPT_TILE_ORDER, FW_OPT_TILE_ROWS)
    case = _case("3d_random_N2_ragged")
    # reference: both updates marching 16-row tiles
    _, ref = _run(case, opts={FW_OPT_TILE_ROWS: 16, FW_OPT_PLANE_KERNELS: 0})
    # (tile rows, rows per thread, chunk, persistent, tile order, plane kernels); a persistent
    # grid keeps the marching kernels.  The 29-plane grid leaves a 1-plane pressure tile.
    for rows, rpt, chunk, pers, order, plane in (
            (4, 1, 0, 0, 0, 1), (8, 1, 8, 0, 0, 0), (8, 2, 13, 1, 0, 1), (16, 2, 0, 0, 0, 0), (16, 1, 9, 2, 0, 1),
            (4, 1, 0, 0, 1, 0), (8, 2, 11, 1, 1, 1), (4, 1, 1, 0, 2, 1), (4, 1, 1, 0, 0, 0), (8, 1, 1, 0, 2, 0),
            (4, 1, 3, 0, 2, 1), (4, 1, 1, 1, 2, 0), (16, 1, 0, 0, 2, 1)):
        opts = {FW_OPT_TILE_ROWS: rows, FW_OPT_ROWS_PER_THREAD: rpt, FW_OPT_PERSISTENT: pers, FW_OPT_TILE_ORDER: order,
                FW_OPT_PLANE_KERNELS: plane}
        if chunk:
            opts[FW_OPT_MARCH_CHUNK] = chunk
        _, got = _run(case, opts=opts)
        assert np.array_equal(ref, got), (rows, rpt, chunk, pers, order, plane)
    # 8-row tiles of the plane kernels (both updates, and pressure only)
    from paper_2606_11103_amd.native import FW_OPT_PLANE_ROWS
    for plane in (1, -1):
        _, got = _run(case, opts={FW_OPT_PLANE_KERNELS: plane, FW_OPT_PLANE_ROWS: 8})
        assert np.array_equal(ref, got), ("plane rows 8", plane)
    # plane-kernel tile depths: 2- and 4-plane velocity tiles, 2/4/8-plane
    # pressure tiles (29 planes: a ragged last tile for each), with 4- and
    # 8-row tiles
    from paper_2606_11103_amd.native import FW_OPT_PRS_PLANES, FW_OPT_VEL_PLANES
    for prow, vp, pp in ((4, 2, 2), (8, 2, 8), (4, 1, 4), (8, 1, 2), (4, 2, 8), (4, 4, 2), (8, 4, 8), (8, 4, 4)):
        _, got = _run(case, opts={FW_OPT_PLANE_KERNELS: 1, FW_OPT_PLANE_ROWS: prow, FW_OPT_VEL_PLANES: vp,
                                  FW_OPT_PRS_PLANES: pp})
        assert np.array_equal(ref, got), ("plane depths", prow, vp, pp)


def test_persistent_grid_on_batched_2d_and_1d():
    from paper_2606_11103_amd.native import FW_OPT_MARCH_CHUNK, FW_OPT_PERSISTENT
    for name in ("2d_batched_N3", "1d_batched_N2"):
        case = _case(name)
        _, ref = _run(case)
        _, got = _run(case, opts={FW_OPT_PERSISTENT: 1, FW_OPT_MARCH_CHUNK: 16})
        assert np.array_equal(ref, got), name


def test_plane_kernels_on_a_ragged_3d_batch():
    """Three 3D domains of different shapes (ragged in x, y and z; y-tile
    counts 5, 10 and 25, so the XCD bands of the plane lists are uneven and
    padded) in one launch, N = 4: plane kernels bitwise equal to the marching
    kernels, and to the FP64 oracle within the bar."""
    from paper_2606_11103_amd.native import FW_OPT_PLANE_KERNELS
    case = configs.random_small(3, [(70, 17, 21), (33, 38, 17), (130, 97, 18)], 4, 3, seed=41, steps=90, pml=4)
    case = configs.with_table(case, *configs.random_relaxation_table(141, case.n_classes, case.nmech))
    _, march = _run(case, opts={FW_OPT_PLANE_KERNELS: 0})
    _, plane = _run(case, opts={FW_OPT_PLANE_KERNELS: 1})
    assert np.array_equal(march, plane)
    ref = oracle_traces(case)
    glob, worst, n = check_traces(plane, ref)
    report("plane kernels, ragged 3D batch of 3, N=4: rel L2 vs FP64 oracle = %.3e, worst receiver %.3e (%d reached)"
           % (glob, worst, n))


def test_interleaved_chunk_schedule_is_bitwise_equal():
    """FW_OPT_STEP_CHUNK: velocity and pressure plane kernels interleaved in
    chunks of C planes (pressure lagging 3 planes) give the same bits as the
    two whole-grid launches, on a ragged 3D batch whose domains end at
    different planes (17, 18 and 21), with chunk sizes that do and do not
    divide them, 1- and 2-plane velocity tiles and 2/8-plane pressure tiles,
    through graph replay and eager steps."""
    from paper_2606_11103_amd.native import (FW_OPT_GRAPH_STEPS, FW_OPT_PLANE_KERNELS, FW_OPT_PRS_PLANES,
                                             FW_OPT_STEP_CHUNK, FW_OPT_VEL_PLANES)
    case = configs.random_small(3, [(70, 17, 21), (33, 38, 17), (130, 97, 18)], 2, 3, seed=44, steps=70, pml=4)
    case = configs.with_table(case, *configs.random_relaxation_table(144, case.n_classes, case.nmech))
    _, ref = _run(case, opts={FW_OPT_PLANE_KERNELS: 1, FW_OPT_STEP_CHUNK: 0})
    for chunk, vp, pp, gs in ((4, 1, 2, 16), (5, 2, 8, 16), (7, 1, 8, 0), (16, 2, 2, 7), (64, 1, 2, 16)):
        _, got = _run(case, opts={FW_OPT_PLANE_KERNELS: 1, FW_OPT_STEP_CHUNK: chunk, FW_OPT_VEL_PLANES: vp,
                                  FW_OPT_PRS_PLANES: pp, FW_OPT_GRAPH_STEPS: gs})
        assert np.array_equal(ref, got), (chunk, vp, pp, gs)


@pytest.mark.parametrize("nmech", [1, 2, 3, 4])
def test_2d_tile_kernels_on_a_ragged_batch(nmech):
    """Five 2D domains of different shapes (widths 70, 33, 130, 64 and 65
    cells: partial last tiles, one exactly full, one a single cell past a
    tile; heights not multiples of any tile height) in one launch: the 2D
    tile kernels with 4-, 8- and 16-row tiles bitwise equal to the marching
    kernels, with and without a strength map, and to the FP64 oracle within
    the bar."""
    from paper_2606_11103_amd.native import FW_OPT_PLANE_KERNELS, FW_OPT_PLANE_ROWS
    shapes = [(70, 21, 1), (33, 38, 1), (130, 97, 1), (64, 61, 1), (65, 19, 1)]
    case = configs.random_small(2, shapes, nmech, 3, seed=50 + nmech, steps=160, pml=5)
    case = configs.with_table(case, *configs.random_relaxation_table(150 + nmech, case.n_classes, case.nmech))
    print("2D tile kernels, N=%d" % nmech, flush=True)
    _, march = _run(case, opts={FW_OPT_PLANE_KERNELS: 0})
    for rows in (4, 8, 16):
        _, tile = _run(case, opts={FW_OPT_PLANE_KERNELS: 1, FW_OPT_PLANE_ROWS: rows})
        assert np.array_equal(march, tile), rows
    _, auto = _run(case)
    assert np.array_equal(march, auto)
    ref = oracle_traces(case)
    glob, worst, n = check_traces(tile, ref)
    report("2D tile kernels, ragged 2D batch of 5, N=%d: rel L2 vs FP64 oracle = %.3e, worst receiver %.3e "
           "(%d reached)" % (nmech, glob, worst, n))
    if nmech == 4:
        smap = configs.with_strength(case, 7, 0.2, 1.0)
        _, march_s = _run(smap, opts={FW_OPT_PLANE_KERNELS: 0})
        _, tile_s = _run(smap, opts={FW_OPT_PLANE_KERNELS: 1, FW_OPT_PLANE_ROWS: 8})
        assert np.array_equal(march_s, tile_s)
        assert not np.array_equal(march_s, march)


def test_default_kernel_choice_with_one_mechanism():
    """N = 1 in 3D: by default both plane kernels (as with option 1);
    bitwise equal to marching both, and to the oracle within the bar."""
    from paper_2606_11103_amd.native import FW_OPT_PLANE_KERNELS
    case = configs.random_small(3, [(70, 17, 21), (130, 97, 18)], 1, 3, seed=43, steps=90, pml=4)
    case = configs.with_table(case, *configs.random_relaxation_table(143, case.n_classes, case.nmech))
    _, march = _run(case, opts={FW_OPT_PLANE_KERNELS: 0})
    _, auto = _run(case)
    _, plane = _run(case, opts={FW_OPT_PLANE_KERNELS: 1})
    assert np.array_equal(march, auto) and np.array_equal(march, plane)
    ref = oracle_traces(case)
    glob, worst, n = check_traces(auto, ref)
    report("default kernels, ragged 3D batch of 2, N=1: rel L2 vs FP64 oracle = %.3e, worst receiver %.3e (%d reached)"
           % (glob, worst, n))


def test_autotuner_keeps_results(tmp_path):
    from paper_2606_11103_amd.autotune import autotune
    case = _case("3d_random_N4")
    _, ref = _run(case)
    sim = to_simulation(case)
    sim.step(20)
    cfg, timings = autotune(sim, steps=2, cache_path=str(tmp_path / "tune.json"))
    assert len(timings) >= 10 and cfg in [__import__("json").loads(k) for k in timings]
    assert sim.get_step() == 20
    sim.step(case.n_steps - 20)
    assert np.array_equal(sim.read_receivers(), ref)


def test_batched_domains_equal_single_runs():
    case = _case("2d_batched_N3")
    _, allr = _run(case)
    for d in range(len(case.shapes)):
        sub = configs.Case(**{**case.__dict__})
        sub.shapes = [case.shapes[d]]
        sub.class_maps = [case.class_maps[d]]
        sub.class_base = [0]
        b = case.class_base[d]
        sl = slice(b, b + 2)
        for f in ("c", "rho", "alpha0", "y", "b_over_a", "kappa", "d", "alpha"):
            setattr(sub, f, getattr(case, f)[sl])
        sm = case.src_domain == d
        rm = case.rec_domain == d
        sub.src_domain = np.zeros(sm.sum(), np.int32)
        sub.src_cell = case.src_cell[sm]
        sub.src_wave = case.src_wave[sm]
        sub.rec_domain = np.zeros(rm.sum(), np.int32)
        sub.rec_cell = case.rec_cell[rm]
        # the stability bound uses the largest speed of all classes in both runs
        sub.pml_params = (1e-4, 1e6, float(case.c.max()))
        case.pml_params = (1e-4, 1e6, float(case.c.max()))
        _, one = _run(sub)
        _, allr = _run(case)
        assert np.array_equal(one, allr[:, rm]), d


def test_save_load_resume_is_bitwise():
    case = _case("2d_random_N4")
    n = case.n_steps
    sim, full = _run(case)
    sim2 = to_simulation(case)
    sim2.step(n // 2)
    buf = sim2.save_state()
    sim2.step(17)                 # advance, then rewind to the snapshot
    sim2.load_state(buf)
    assert sim2.get_step() == n // 2
    sim2.step(n - n // 2)
    assert np.array_equal(sim2.read_receivers(), full)


def test_reset_reproduces_first_run():
    case = _case("2d_random_N1_linear")
    sim, a = _run(case)
    sim.reset()
    sim.step(case.n_steps)
    assert np.array_equal(sim.read_receivers(), a)


@pytest.mark.parametrize("nmech", [1, 2, 3, 4])
def test_resident_1d_step_equals_the_per_step_kernels(nmech):
    """FW_OPT_RESIDENT_1D: a ragged 1D batch (8192 cells, the largest domain
    kept on chip, then 3001 and 77) with per-cell classes, speed perturbation,
    nonlinear media, CPML and receivers on every domain's first and last
    cells, stepped in calls of 1, 99, 4200 (two launches of the resident
    kernel) and the rest: traces and the whole saved state (every field and
    memory variable, the step counter and the finite-check row) bitwise equal
    to the per-step kernels, and the traces within the bar of the FP64
    oracle."""
    import torch
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    case = configs.random_small(1, [(8192, 1, 1), (3001, 1, 1), (77, 1, 1)], nmech, 3, seed=60 + nmech, steps=4500,
                                pml=24)
    case = configs.with_table(case, *configs.random_relaxation_table(150 + nmech, case.n_classes, case.nmech))
    case.rec_domain = np.concatenate([case.rec_domain, np.repeat(np.arange(3, dtype=np.int32), 2)])
    case.rec_cell = np.concatenate([case.rec_cell, np.array([0, 8191, 0, 3000, 0, 76], np.int64)])
    print("resident 1D", case.shapes, "N=%d" % nmech, flush=True)
    ref_sim, ref = _run(case, opts={FW_OPT_RESIDENT_1D: 0})
    sim = to_simulation(case)
    sim.prepare()
    for n in (1, 99, 4200, case.n_steps - 4300):
        sim.step(n)
    assert sim.get_step() == case.n_steps
    got = sim.read_receivers()
    assert np.array_equal(ref, got)
    # a snapshot holds the state and then the step counter and the finite-check row
    used = sim.state_bytes() - 256 + 16
    assert torch.equal(sim.save_state()[:used], ref_sim.save_state()[:used])
    glob, worst, n = check_traces(got, oracle_traces(case))
    report("resident 1D N=%d %s: bitwise equal to the per-step kernels; rel_L2=%.3e worst_receiver=%.3e (%d reached)"
           % (nmech, case.shapes, glob, worst, n))


@pytest.mark.parametrize("nmech,noise", [(1, 0.0), (2, 0.0), (2, 0.01), (4, 0.0)])
def test_resident_1d_single_class_domains(nmech, noise):
    """Domains of one tissue class each (as in the attenuation sweep), which
    the resident step runs with every coefficient held in scalar registers
    at N <= 2 when the speed perturbation is off: bitwise equal to the
    per-step kernels over 4200 steps (two launches)."""
    import torch
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    case = configs.random_small(1, [(8192, 1, 1), (5000, 1, 1), (64, 1, 1)], nmech, 1, seed=90 + nmech, steps=4200,
                                pml=24, noise=noise)
    case = configs.with_table(case, *configs.random_relaxation_table(190 + nmech, case.n_classes, case.nmech))
    ref_sim, ref = _run(case, opts={FW_OPT_RESIDENT_1D: 0})
    sim, got = _run(case)
    assert np.array_equal(ref, got)
    used = sim.state_bytes() - 256 + 16
    assert torch.equal(sim.save_state()[:used], ref_sim.save_state()[:used])


def test_resident_1d_path_is_the_one_taken():
    """The resident comparisons above only mean something if the default
    really runs the resident kernel: on 256 domains of 8192 cells it is
    several times faster than the per-step kernels (about 9x measured), which
    no other path reaches."""
    import torch
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    case = configs.random_small(1, [(8192, 1, 1)] * 256, 2, 1, seed=5, steps=2000, pml=24, noise=0.0)
    case = configs.with_table(case, *configs.random_relaxation_table(5, case.n_classes, case.nmech))
    ms = {}
    for resident in (0, -1):
        sim = to_simulation(case)
        sim.set_option(FW_OPT_RESIDENT_1D, resident)
        sim.prepare()
        sim.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(case.n_steps - 10)
        torch.cuda.synchronize()
        ms[resident] = 1e3 * (time.perf_counter() - t0)
    report("resident 1D, 256 x 8192 cells, N=2, %d steps: %.1f ms resident, %.1f ms per-step kernels"
           % (case.n_steps - 10, ms[-1], ms[0]))
    assert 3.0 * ms[-1] < ms[0]


def test_resident_1d_mixed_with_energy_steps_and_rewind():
    """Resident launches interleaved with energy steps (which take the
    per-step kernels), an odd number of steps between them, and a rewind to a
    saved state: traces, energies and the final state bitwise equal to the
    same sequence run with the per-step kernels only."""
    import torch
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    case = configs.random_small(1, [(4096, 1, 1), (999, 1, 1)], 3, 3, seed=311, steps=900, pml=16)
    case = configs.with_table(case, *configs.random_relaxation_table(311, case.n_classes, case.nmech))
    out = []
    for resident in (0, -1):
        sim = to_simulation(case)
        sim.set_option(FW_OPT_RESIDENT_1D, resident)
        energies = []
        sim.step(101)
        energies.append(sim.energy_step())
        sim.step(250)
        snap = sim.save_state()
        sim.step(33)
        energies.append(sim.energy_step())
        sim.load_state(snap)
        assert sim.get_step() == 352
        energies.append(sim.energy_step())
        sim.step(case.n_steps - 353)
        assert sim.get_step() == case.n_steps
        used = sim.state_bytes() - 256 + 16
        out.append((sim.read_receivers(), np.stack(energies), sim.save_state()[:used]))
    (ref, e_ref, s_ref), (got, e_got, s_got) = out
    assert np.array_equal(ref, got)
    assert np.array_equal(e_ref, e_got)
    assert torch.equal(s_ref, s_got)
    glob, worst, n = check_traces(got, oracle_traces(case))
    report("resident 1D mixed with energy steps and a rewind: bitwise equal; rel_L2=%.3e worst_receiver=%.3e "
           "(%d reached)" % (glob, worst, n))


def test_resident_1d_flags_the_first_non_finite_row():
    """A finite source sample that overflows p: the resident 1D step records
    the first trace row holding a non-finite value, as the per-step kernels
    do, across several domains advancing in separate workgroups."""
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    case = configs.random_small(1, [(700, 1, 1), (300, 1, 1)], 2, 2, seed=77, steps=60, nonlinear=False)
    case = configs.with_table(case, *configs.random_relaxation_table(77, case.n_classes, case.nmech))
    case.waves = case.waves.copy()
    case.waves[0, 20] = np.float32(3e38)
    case.waves[0, 21] = np.float32(3e38)
    ref_sim, ref = _run(case, opts={FW_OPT_RESIDENT_1D: 0})
    sim, got = _run(case)
    bad = np.nonzero(~np.all(np.isfinite(got), axis=1))[0]
    assert bad.size > 0
    assert np.array_equal(np.isfinite(ref), np.isfinite(got))
    assert sim.first_nonfinite_step() == ref_sim.first_nonfinite_step() == bad[0]


def test_resident_1d_before_any_source_or_receiver():
    """A 1D batch stepped before any source or receiver is set: the resident
    step runs without a per-domain source/receiver table, the field stays
    zero, and the state then equals the per-step kernels' bit for bit."""
    import torch
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    from paper_2606_11103_amd.sim import Simulation
    kappa, d, al = configs.random_relaxation_table(5, 2, 2)
    sims = []
    for resident in (-1, 0):
        sim = Simulation(1, [(500, 1, 1), (300, 1, 1)], 1e-4, 2e-8, 2, 10)
        sim.set_option(FW_OPT_RESIDENT_1D, resident)
        sim.set_media([np.zeros(500, np.uint8), np.zeros(300, np.uint8)], [0, 1], [1500.0, 1550.0], [1000.0, 1050.0],
                      [0.0, 0.0])
        sim.set_relaxation_table(kappa, d, al)
        sim.step(77)
        assert sim.get_step() == 77
        assert np.all(sim.read_field(0, 0) == 0.0) and np.all(sim.read_field(0, 1) == 0.0)
        sims.append(sim)
    used = sims[0].state_bytes() - 256 + 16
    assert torch.equal(sims[0].save_state()[:used], sims[1].save_state()[:used])
