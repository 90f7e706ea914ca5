"""Edge cases of the HIP path against the FP64 oracle: no sources, a closed
box without CPML, the smallest admissible domains in a ragged batch,
sources and receivers on the grid's corners and faces, repeated receivers."""
import zlib

import numpy as np
import pytest

from workloads import configs, linear_index
from workloads.adapters import oracle_traces, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu


def _tables(case, name):
    return configs.with_table(case, *configs.random_relaxation_table(zlib.crc32(name.encode()) % 1000,
                                                                     case.n_classes, case.nmech))


def _parity(case, name):
    print("edge case", name, case.shapes, flush=True)
    sim = to_simulation(case)
    sim.step(case.n_steps)
    got = sim.read_receivers().astype(np.float64)
    ref = oracle_traces(case)
    glob, worst, n = check_traces(got, ref)
    report("edge %s rel_L2=%.3e worst_receiver=%.3e (%d of %d reached) steps=%d"
           % (name, glob, worst, n, len(case.rec_cell), case.n_steps))
    return got


def test_without_sources_the_field_stays_zero():
    case = _tables(configs.random_small(3, [(30, 28, 26)], 2, 2, seed=5, steps=40), "nosrc")
    case.src_domain = case.src_domain[:0]
    case.src_cell = case.src_cell[:0]
    case.src_wave = case.src_wave[:0]
    sim = to_simulation(case)
    sim.step(39)
    e = sim.energy_step()[0]
    assert e[0] == 0.0 and e[1] == 0.0 and e[2] == 0
    assert np.all(sim.read_receivers() == 0.0)


def test_closed_box_without_cpml():
    case = _tables(configs.random_small(2, [(90, 70, 1)], 3, 3, seed=12, steps=300, pml=0), "nopml")
    _parity(case, "no_cpml_2d")


def test_smallest_domains_in_a_ragged_batch():
    """Every used dimension at its minimum, 2 P + 9 (P = 4), next to larger
    domains of the same batch, in 3D and 1D."""
    P = 4
    m = 2 * P + 9
    case = _tables(configs.random_small(3, [(m, m, m), (m + 13, m, m + 2), (m, m + 21, m)], 2, 2, seed=14,
                                        steps=60, pml=P), "min3d")
    _parity(case, "smallest_3d")
    case = _tables(configs.random_small(1, [(m, 1, 1), (m + 1, 1, 1), (64, 1, 1)], 3, 2, seed=15, steps=80,
                                        pml=P), "min1d")
    _parity(case, "smallest_1d")


def test_sources_and_receivers_on_corners_and_faces():
    """Point sources in two opposite corners (inside the CPML) and receivers
    on every face, corner and edge; one receiver cell listed three times."""
    shp = (37, 31, 29)
    case = _tables(configs.random_small(3, [shp], 2, 3, seed=16, steps=90, pml=5, amplitude=3e5), "corners")
    nx, ny, nz = shp
    src = [linear_index(shp, 0, 0, 0), linear_index(shp, nx - 1, ny - 1, nz - 1)]
    case.src_domain = np.zeros(2, np.int32)
    case.src_cell = np.array(src, np.int64)
    case.src_wave = np.zeros(2, np.int32)
    rec = [linear_index(shp, x, y, z) for x in (0, nx // 2, nx - 1) for y in (0, ny - 1) for z in (0, nz // 3, nz - 1)]
    rec += [linear_index(shp, 1, 1, 1)] * 3
    case.rec_domain = np.zeros(len(rec), np.int32)
    case.rec_cell = np.array(rec, np.int64)
    got = _parity(case, "corners_faces_3d")
    assert np.array_equal(got[:, -1], got[:, -2]) and np.array_equal(got[:, -1], got[:, -3])


def test_many_sources_and_receivers_over_several_workgroups():
    """A 1D batch of 60 domains, each with a source and 6 receivers: one on
    the source cell (it records the injected value), one listed twice and
    three more, 300 distinct cells, so the source/receiver step spans
    several workgroups (256 cells each). Against the FP64 oracle; the step
    counter stays right over graph replays and eager steps."""
    from paper_2606_11103_amd.native import FW_OPT_GRAPH_STEPS
    shapes = [(160 + 7 * d, 1, 1) for d in range(60)]
    case = _tables(configs.random_small(1, shapes, 2, 2, seed=77, steps=120, pml=6, n_rec=1), "many_srcrec")
    rd, rc = [], []
    for d, (n, _, _) in enumerate(shapes):
        s = int(case.src_cell[d])
        for c in (s, n // 3, n // 3, n // 2, 2 * n // 3, n - 1):
            rd.append(d)
            rc.append(c)
    case.rec_domain = np.array(rd, np.int32)
    case.rec_cell = np.array(rc, np.int64)
    assert len(set(zip(rd, rc))) > 256 and len(case.src_cell) == 60
    got = _parity(case, "many_sources_receivers_1d")
    assert np.array_equal(got[:, 1::6], got[:, 2::6])          # the repeated receiver
    # graph replays (7 steps per graph) and eager steps give the same traces and counter
    sim = to_simulation(case)
    sim.set_option(FW_OPT_GRAPH_STEPS, 7)
    sim.step(50)
    sim.set_option(FW_OPT_GRAPH_STEPS, 0)
    sim.step(case.n_steps - 50)
    assert sim.get_step() == case.n_steps
    assert np.array_equal(sim.read_receivers(), got.astype(np.float32))


def test_receivers_into_a_caller_buffer():
    """fw_set_receivers_into: the traces land in the caller's device tensor,
    bit for bit the library-buffer traces; read-back and reset use it; once
    receivers are set again with the library's buffer the tensor is no longer
    written."""
    import torch
    case = _tables(configs.random_small(2, [(70, 50, 1), (40, 45, 1)], 3, 2, seed=71, steps=120, pml=6), "into")
    ref_sim = to_simulation(case)
    ref_sim.step(case.n_steps)
    ref = ref_sim.read_receivers()
    sim = to_simulation(case)
    n_rec = len(case.rec_cell)
    buf = torch.full((case.n_steps + 5, n_rec), 7.0, dtype=torch.float32, device=sim.device)   # larger than needed
    sim.set_receivers(case.rec_domain, case.rec_cell, case.n_steps, out=buf)
    assert float(buf[: case.n_steps].abs().max()) == 0.0          # zeroed by the library
    sim.step(case.n_steps)
    torch.cuda.synchronize()
    got = buf[: case.n_steps].cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(sim.read_receivers(), ref)
    assert float(buf[case.n_steps:].sub(7.0).abs().max()) == 0.0   # past the traces: untouched
    sim.reset()
    torch.cuda.synchronize()
    assert float(buf[: case.n_steps].abs().max()) == 0.0
    sim.set_receivers(case.rec_domain, case.rec_cell, case.n_steps)
    buf.fill_(3.0)
    sim.step(10)
    torch.cuda.synchronize()
    assert float(buf.sub(3.0).abs().max()) == 0.0
    with pytest.raises(Exception):
        sim.set_receivers(case.rec_domain, case.rec_cell, case.n_steps,
                          out=torch.zeros(case.n_steps * n_rec - 1, dtype=torch.float32, device=sim.device))
