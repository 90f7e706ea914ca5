"""Parity at full size.

The 2D two-layer workload (2048 x 2048, N = 4, nonlinear, 4000 steps) is
compared over every receiver and step with the FP64 oracle's traces, stored
under tests/golden by a script that runs only the oracle (the oracle needs
minutes of host time for it); the inputs stored with them (tables, speeds,
cells, waveform) are checked against the workload generator first.

The 960 x 960 x 720 workload (N = 4, 24-cell CPML, 8 classes, speed
perturbation, nonlinear, focused array) is run on the GPU exactly as
bench.py runs it.  After K steps the field is provably zero farther than
8 K cells from the sources (each step's two stencils reach 4 cells each), so
the FP64 oracle on the box that contains that support computes the same
field; every pressure value of the box and every receiver inside it is
compared, and the GPU field outside the box must be exactly zero.
"""
import os

import numpy as np
import pytest

from workloads import configs
from workloads.adapters import to_oracle_crop, to_simulation
from reporting import report
from parity_metrics import check_traces

pytestmark = pytest.mark.gpu


def _support_parity(case, K, label):
    """Run K steps on the GPU; every pressure of the box holding the field's
    support and every receiver inside it against the FP64 oracle on that box
    (relative L2 <= 1e-5), and exact zeros outside the box."""
    print(label, case.shapes, "steps", K, flush=True)
    sim = to_simulation(case)
    sim.step(K)
    p = sim.read_field(0)
    traces = sim.read_receivers()[:K]
    del sim
    nx, ny, nz = case.shapes[0]
    sx = case.src_cell % nx
    sy = (case.src_cell // nx) % ny
    sz = case.src_cell // (nx * ny)
    m = 8 * K + 8
    lo = [max(0, int(sx.min()) - m), max(0, int(sy.min()) - m), max(0, int(sz.min()) - m)]
    hi = [min(nx, int(sx.max()) + 1 + m), min(ny, int(sy.max()) + 1 + m), min(nz, int(sz.max()) + 1 + m)]
    box = p[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].astype(np.float64)
    outside_max = 0.0
    for (z0, z1) in ((0, lo[2]), (hi[2], nz)):
        if z1 > z0:
            outside_max = max(outside_max, float(np.abs(p[z0:z1]).max()))
    sl = p[lo[2]:hi[2]]
    for part in (sl[:, :lo[1]], sl[:, hi[1]:], sl[:, lo[1]:hi[1], :lo[0]], sl[:, lo[1]:hi[1], hi[0]:]):
        if part.size:
            outside_max = max(outside_max, float(np.abs(part).max()))
    del p, sl
    assert outside_max == 0.0

    orc = to_oracle_crop(case, lo, hi)
    lx, ly = hi[0] - lo[0], hi[1] - lo[1]
    local = ((sz - lo[2]) * ly + (sy - lo[1])) * lx + (sx - lo[0])
    rx = case.rec_cell % nx
    ry = (case.rec_cell // nx) % ny
    rz = case.rec_cell // (nx * ny)
    inside = (rx >= lo[0]) & (rx < hi[0]) & (ry >= lo[1]) & (ry < hi[1]) & (rz >= lo[2]) & (rz < hi[2])
    rloc = ((rz - lo[2]) * ly + (ry - lo[1])) * lx + (rx - lo[0])
    rec, _ = orc.run(K, local, case.waves.astype(np.float64)[case.src_wave], rloc[inside])
    ref = orc.p.reshape(box.shape)
    rel_field = float(np.linalg.norm(box - ref) / np.linalg.norm(ref))
    rel_rec = float(np.linalg.norm(traces[:, inside] - rec) / np.linalg.norm(rec))
    report("%s %s N=%d after %d steps: box %s rel_L2 field=%.3e receivers(%d)=%.3e"
           % (label, "x".join(str(n) for n in case.shapes[0]), case.nmech, K, [h - l for l, h in zip(lo, hi)],
              rel_field, int(inside.sum()), rel_rec))
    assert rel_field <= 1e-5 and rel_rec <= 1e-5


def test_full_size_3d_workload_matches_oracle_on_the_field_support():
    from paper_2606_11103_amd import relax
    case = configs.heterogeneous_3d(shape=(960, 960, 720), steps=2000)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    _support_parity(case, 10, "full-size 3D")


def test_largest_admissible_domain_matches_oracle_on_the_field_support():
    """1280^3 = 2.097e9 cells, just under the 2^31 cells a domain may hold
    (in-domain offsets are 32-bit), with the same recipe at N = 2 (about
    153 GB of state).  Sources and receivers are mirrored to the last planes
    (z -> nz - 1 - z), so the checked support sits at the top of the 32-bit
    offset range."""
    import torch
    torch.cuda.empty_cache()
    case = configs.heterogeneous_3d(shape=(1280, 1280, 1280), steps=64, nmech=2)
    assert case.cells() < 2 ** 31 and case.cells() > 2 ** 31 - 2 ** 28
    nx, ny, nz = case.shapes[0]
    for name in ("src_cell", "rec_cell"):
        c = getattr(case, name)
        z = c // (nx * ny)
        setattr(case, name, (c - z * nx * ny + (nz - 1 - z) * nx * ny).astype(np.int64))
    assert int(case.src_cell.min()) > case.cells() - 2 ** 26
    configs.with_table(case, *configs.random_relaxation_table(1280, case.n_classes, case.nmech))
    _support_parity(case, 6, "largest domain 3D")
    torch.cuda.empty_cache()


GOLDEN_2D = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_layer_2d_2048_oracle.npz")


def test_full_size_two_layer_2d_matches_stored_oracle_traces():
    g = np.load(GOLDEN_2D)
    steps = int(g["steps"])
    case = configs.two_layer_2d(steps=steps)
    # the stored inputs are the workload's
    np.testing.assert_array_equal(g["c"], case.c)
    np.testing.assert_array_equal(g["rho"], case.rho)
    np.testing.assert_array_equal(g["rec_cell"], case.rec_cell)
    np.testing.assert_array_equal(g["src_cell"], case.src_cell)
    np.testing.assert_array_equal(g["wave"], case.waves[0])
    assert float(g["dx"]) == case.dx and float(g["dt"]) == case.dt
    configs.with_table(case, g["kappa"], g["d"], g["alpha"])
    print("full-size 2D two-layer", case.shapes, "steps", steps, flush=True)
    sim = to_simulation(case)
    sim.step(steps)
    tr = sim.read_receivers()[:steps].astype(np.float64)
    del sim
    ref = g["traces"].astype(np.float64)
    zero = np.linalg.norm(ref, axis=0) == 0
    assert np.all(tr[:, zero] == 0.0)
    rel, worst, n = check_traces(tr, ref)
    report("full-size 2D two-layer 2048x2048 N=4 nonlinear, %d steps x %d receivers (%d reached): rel_L2 %.3e "
           "(worst receiver %.3e), peak |p| %.3g Pa" % (steps, tr.shape[1], n, rel, worst, np.abs(ref).max()))


def test_full_size_3d_run_is_finite_and_loses_energy_after_the_source():
    """All 2000 steps of the benchmark workload: every pressure stays finite,
    and once the source has ended (its pulses are over by step ~200) the FP64
    staggered-time energy only decreases (attenuation, CPML absorption)."""
    from paper_2606_11103_amd import relax
    case = configs.heterogeneous_3d(shape=(960, 960, 720), steps=2000)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    print("full-size 3D, 2000 steps", flush=True)
    sim = to_simulation(case)
    marks = (400, 800, 1200, 1600, 2000)
    energy = []
    done = 0
    for m in marks:
        sim.step(m - 1 - done)
        e = sim.energy_step()[0]
        done = m
        assert e[2] == 0
        energy.append((m, e[0], e[1]))
    tr = sim.read_receivers()
    del sim
    report("full-size 3D 2000 steps: energy/max|p| at steps " +
            ", ".join("%d: E %.3e, %.3g Pa" % v for v in energy))
    assert np.all(np.isfinite(tr))
    E = [v[1] for v in energy]
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))


def test_full_size_batched_2d_equals_single_shots():
    """The 64 ragged shots of the batched benchmark (one tile list) give
    bit-identical traces to the same shots run as simulations of their own."""
    case = configs.batched_2d(steps=40)
    configs.with_table(case, *configs.random_relaxation_table(4000, case.n_classes, case.nmech))
    case.pml_params = (1e-4, 1e6, float(case.c.max()))
    sim = to_simulation(case)
    sim.step(40)
    allr = sim.read_receivers()
    del sim
    for s in (0, 37, 63):
        one = configs.Case(**{**case.__dict__})
        one.shapes = [case.shapes[s]]
        one.class_maps = [case.class_maps[s]]
        one.class_base = [0]
        b = case.class_base[s]
        sl = slice(b, b + int(case.class_maps[s].max()) + 1)
        for f in ("c", "rho", "alpha0", "y", "b_over_a", "kappa", "d", "alpha"):
            setattr(one, f, getattr(case, f)[sl])
        sm = case.src_domain == s
        rm = case.rec_domain == s
        one.src_domain = np.zeros(int(sm.sum()), np.int32)
        one.src_cell = case.src_cell[sm]
        one.src_wave = case.src_wave[sm]
        one.rec_domain = np.zeros(int(rm.sum()), np.int32)
        one.rec_cell = case.rec_cell[rm]
        sim = to_simulation(one)
        sim.step(40)
        r = sim.read_receivers()
        del sim
        assert np.array_equal(r, allr[:, rm]), s


def test_full_size_adjoint_is_independent_of_the_checkpoint_interval():
    """The 1024 x 1024 x 16-shot adjoint workload over 110 steps: gradients
    with checkpoints every 55 steps and every 22 steps are bit-identical and
    finite."""
    import torch
    case = configs.adjoint_2d(steps=110)
    from paper_2606_11103_amd import relax
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    sim = to_simulation(case)
    out = []
    for ck in (55, 22):
        work = sim.adjoint_workspace(110, ck)
        sim.forward_checkpointed(110, ck, work)
        tr = sim.read_receivers_device()
        gK, gs = sim.adjoint_modulus(110, ck, work, case.dt * tr)
        out.append((gK.cpu().numpy(), gs.cpu().numpy()))
        del work
        torch.cuda.empty_cache()
    del sim
    assert np.all(np.isfinite(out[0][0])) and np.all(np.isfinite(out[0][1]))
    assert np.abs(out[0][0]).max() > 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_full_size_3d_state_round_trip_is_bitwise():
    """The 960 x 960 x 720, N = 4 state (about 69 GB) is larger than one
    copy launch can cover (2^32 lanes of 16 bytes): a snapshot taken after 40
    steps, restored after 3 more, gives the same next step bit for bit in
    every field, and the step counter comes back with it."""
    import torch
    from paper_2606_11103_amd import relax
    torch.cuda.empty_cache()
    case = configs.heterogeneous_3d(shape=(960, 960, 720), steps=2000)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    print("full-size 3D state round trip", case.shapes, flush=True)
    sim = to_simulation(case)
    assert sim.state_bytes() > 16 * 2 ** 32
    sim.step(40)
    buf = sim.save_state()
    sim.step(1)
    ref = [sim.read_field(f, device=True) for f in range(4)]
    assert float(ref[0].abs().max()) > 0.0
    sim.step(2)
    sim.load_state(buf)
    assert sim.get_step() == 40
    sim.step(1)
    same = [bool(torch.equal(sim.read_field(f, device=True), ref[f])) for f in range(4)]
    report("full-size 3D state round trip (%.1f GB): fields bitwise equal %s" % (sim.state_bytes() / 1e9, same))
    del sim, buf, ref
    torch.cuda.empty_cache()
    assert all(same)


def test_full_size_interleaved_schedule_equals_whole_grid_launches():
    """On the 960 x 960 x 720, N = 4 grid the step runs by default as
    interleaved velocity/pressure chunks of 120 planes (pressure lagging 3
    planes); 60 steps of it give the same pressure and velocity fields, bit for
    bit, as 60 steps of the two whole-grid launches (FW_OPT_STEP_CHUNK 0)."""
    import torch
    from paper_2606_11103_amd import relax
    from paper_2606_11103_amd.native import FW_OPT_STEP_CHUNK
    torch.cuda.empty_cache()
    case = configs.heterogeneous_3d(shape=(960, 960, 720), steps=2000)
    kappa, d, al, _ = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                      allow_fit=False, dt=case.dt)
    configs.with_table(case, kappa, d, al)
    print("full-size 3D interleaved schedule", case.shapes, flush=True)
    sim = to_simulation(case)
    sim.set_option(FW_OPT_STEP_CHUNK, 0)
    sim.step(60)
    ref = [sim.read_field(f, device=True) for f in range(4)]
    del sim
    torch.cuda.empty_cache()
    assert float(ref[0].abs().max()) > 0.0
    sim = to_simulation(case)
    sim.step(60)
    same = [bool(torch.equal(sim.read_field(f, device=True), ref[f])) for f in range(4)]
    report("full-size 3D interleaved chunks vs whole-grid launches, 60 steps: fields bitwise equal %s" % (same,))
    del sim, ref
    torch.cuda.empty_cache()
    assert all(same)
