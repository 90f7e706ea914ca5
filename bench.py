"""Benchmark of the FDTD step on one MI355X.

Workload: the 3D heterogeneous case -- 960 x 960 x 720 cells, dx = 0.1 mm,
8 tissue classes from a seeded smoothed label field, +-1 % per-voxel speed
perturbation, N = 4 relaxation mechanisms, 24-cell CPML, nonlinear, focused
64-element source (synthetic data; relaxation tables from the FP64
calibration).  A "step" is one full time step: velocity update, pressure
update, sources and receivers.

Prints one JSON line: Gcell-updates/s of the whole job timed through the
graph-replayed step, the HBM roofline fraction of the whole step (with the
dominant kernel, the velocity update, and the pressure update as sub-fields
from a separate per-kernel pass), and the FP64 oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Counted bytes of the benchmark's kernels measured with rocprofv3 --pmc
# (FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000 per dispatch, factors from the
# library's plain copy kernel): per step, of all kernels of one step and of
# its velocity launches, keyed by the SHA-256 prefix of the kernel sources they
# were taken on and by the step's schedule (planes per chunk of the interleaved
# schedule, 0 for whole-grid launches); any other kernel source or schedule
# reports traffic as null.
TRAFFIC_MEASURED = {
    # velocity plane kernel (64 x 4 tiles, 1 plane) + pressure plane kernel (64 x 4
    # tiles, 2 planes) + sources/receivers, in 6 interleaved chunks of 120 planes
    # per step; FETCH_SIZE counts L2 misses sent to the data fabric, so the
    # z-window reads served by the last-level cache are included: an upper bound
    # on the HBM bytes
    ("567f6cbf917326a1", 120): {"workload": "3d_heterogeneous_960x960x720", "step_bytes": 144.85e9,
                                "velocity_bytes": 99.30e9,
                                "profile": "profiles/step_kernels_3d_960x960x720_N4.md"},
}

# The library's automatic choice of the interleaved schedule (FW_OPT_STEP_CHUNK
# -1): 3D grids with both plane kernels, at least 320 planes and a plane of at
# least 100 k cells run 120-plane chunks.
AUTO_CHUNK, AUTO_CHUNK_MIN_PLANES, AUTO_CHUNK_MIN_PLANE_CELLS = 120, 320, 100000


def step_chunk_planes(case, step_chunk=None, plane_kernels=None):
    """Planes per chunk of the step's interleaved schedule for this case,
    FW_OPT_STEP_CHUNK value (None: the default) and FW_OPT_PLANE_KERNELS value
    (None: the default, plane kernels in 3D), 0 for whole-grid launches."""
    if case.ndim != 3 or step_chunk == 0 or plane_kernels == 0:
        return 0
    if step_chunk is not None and step_chunk > 0:
        return int(step_chunk)
    nz = max(int(s[2]) for s in case.shapes)
    plane = max(int(s[0]) * int(s[1]) for s in case.shapes)
    return AUTO_CHUNK if nz >= AUTO_CHUNK_MIN_PLANES and plane >= AUTO_CHUNK_MIN_PLANE_CELLS else 0


def kernel_source_hash():
    """SHA-256 prefix of the step kernels' sources (the kernel file and the two
    headers it includes: argument structures and device helpers)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("fw_kernels.hip", "fw_internal.h", "fw_vec.h"):
        with open(os.path.join(ROOT, "paper_2606_11103_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(case):
    """Algorithmic bytes per cell-update (FP32 state read once and written
    once, uint8 class index, CPML variables inside the slabs):
      velocity kernel: p (4) + class (1) + v r/w (8 ndim) + psi1 r/w (8 N ndim)
                       + CPML face variable r/w (8) per slab axis
      pressure kernel: v (4 ndim) + p r/w (8) + psi2 r/w (8 N) + class (1)
                       + CPML cell variable r/w (8) per slab axis
      whole step (minimum of any schedule): every state float read and written
                       once, class read once: (1 + ndim + N (ndim + 1)) 8 + 1
                       + 16 per slab axis."""
    nd, N, P = case.ndim, case.nmech, case.pml_cells
    cells = case.cells()
    slab = 0.0
    for shp in case.shapes:
        c = float(np.prod(shp))
        for a in range(nd):
            slab += c * min(1.0, 2.0 * P / shp[a])
    slab_frac = slab / cells           # sum over axes of the slab fraction
    vel = 4 + 1 + 8 * nd + 8 * N * nd + 8 * slab_frac
    prs = 4 * nd + 8 + 8 * N + 1 + 8 * slab_frac
    step = (1 + nd + N * (nd + 1)) * 8 + 1 + 16 * slab_frac
    return vel, prs, step


def bench_case(full=True, shape=None, nmech=4):
    """The benchmark workload (3D heterogeneous recipe, 960 x 960 x 720, N = 4);
    shape / nmech select the same recipe on another grid or mechanism count
    (profiling runs, not the benchmark)."""
    from workloads import configs
    if shape is None:
        shape = (960, 960, 720) if full else (192, 160, 128)
    return configs.heterogeneous_3d(shape=tuple(shape), steps=2000, nmech=nmech)


def fill_tables(case, allow_fit=True):
    from paper_2606_11103_amd import relax
    classes = dict(c=case.c, alpha0=case.alpha0, y=case.y)
    kappa, d, al, fits = relax.tables_for(classes, case.nmech, allow_fit=allow_fit, dt=case.dt)
    case.kappa, case.d, case.alpha = kappa, d, al
    return fits


def cpu_baseline(seconds_target=20.0, gpu=False):
    """The FP64 oracle as it stands, on a 128 x 128 x 96 crop-sized instance of
    the same recipe (same classes, tables, noise, source), timed on the host;
    with gpu, the library then runs the same instance for the same steps and
    its receiver traces are compared with the oracle's ("parity")."""
    from workloads import configs
    from workloads.adapters import to_oracle
    case = configs.heterogeneous_3d(shape=(128, 128, 96), steps=2000, n_elem=16)
    fill_tables(case)
    sim = to_oracle(case)
    waves = case.waves.astype(np.float64)[case.src_wave]
    steps = 0
    traces = []
    t0 = time.perf_counter()
    while True:
        rec, _ = sim.run(10, case.src_cell, waves, case.rec_cell)
        traces.append(np.asarray(rec, np.float64))
        steps += 10
        el = time.perf_counter() - t0
        if el >= seconds_target or steps >= 2000:
            break
    cells = case.cells()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    out = dict(value=cells * steps / el / 1e9, unit="Gcell-updates/s", cores=cores, kind="oracle",
               sample="FP64 oracle, 128x128x96 instance of the 3D heterogeneous recipe (N=4, CPML 24, "
                      "noise, nonlinear), %d steps in %.1f s" % (steps, el))
    if gpu:
        # the library on the same instance and steps, against the oracle's traces
        from workloads.adapters import to_simulation
        ref = np.concatenate(traces)[:steps]
        lib = to_simulation(case)
        lib.step(steps)
        got = lib.read_receivers()[:steps].astype(np.float64)
        del lib
        out["parity"] = dict(zip(("rel_l2", "worst_receiver_rel_l2", "receivers_reached"),
                                 trace_errors(got, ref)), steps=steps)
    return out


def trace_errors(got, ref, reach=1e-3):
    """Relative L2 of the receiver traces [steps][receivers] over all of them,
    the worst relative L2 of one receiver among those whose peak reaches
    `reach` of the strongest, and the number of those receivers."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    glob = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    peak = np.abs(ref).max(axis=0)
    reached = peak >= reach * max(peak.max(), 1e-300)
    worst = 0.0
    for r in np.nonzero(reached)[0]:
        worst = max(worst, float(np.linalg.norm(got[:, r] - ref[:, r]) / np.linalg.norm(ref[:, r])))
    return round(glob, 10), round(worst, 10), int(reached.sum())


def bench_record(out, kernel_hash):
    """One JSONL record of a benchmark run: a hash of its configuration, the
    throughput, the roofline figures, the oracle beside it and the parity of
    the oracle's sample."""
    import datetime
    import hashlib
    import platform
    cfg = json.dumps(out.get("config", {}), sort_keys=True)
    r = out.get("roofline", {})
    cb = out.get("cpu_baseline") or {}
    return {
        "time": datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds"),
        "host": platform.node(),
        "config_hash": hashlib.sha256(cfg.encode()).hexdigest()[:16],
        "kernel_source_hash": kernel_hash,
        "workload": out.get("config", {}).get("workload"),
        "metric": out.get("metric"), "value": out.get("value"), "unit": out.get("unit"),
        "ms_per_step": out.get("ms_per_step"),
        "roofline_frac": r.get("frac"), "algorithmic_GBps": r.get("achieved"), "counted_GBps": r.get("traffic"),
        "dominant_kernel_frac": (r.get("dominant_kernel") or {}).get("frac"),
        "oracle_gcells": cb.get("value"), "oracle_cores": cb.get("cores"),
        "parity": cb.get("parity"),
    }


def oracle_timings(seconds=8.0):
    """The FP64 oracle (as it stands) on bounded samples of each workload, in
    Gcell-updates/s of that sample; for reporting beside the GPU figures."""
    from workloads import configs
    from workloads.adapters import to_oracle

    def timed(case, domains, label):
        cells, steps_done, t_all = 0, 0, 0.0
        for d in domains:
            sim = to_oracle(case, d)
            sm = case.src_domain == d
            waves = case.waves.astype(np.float64)[case.src_wave[sm]]
            rm = np.nonzero(case.rec_domain == d)[0]
            n = 0
            t0 = time.perf_counter()
            while n < case.n_steps and time.perf_counter() - t0 < seconds / len(domains):
                sim.run(10, case.src_cell[sm], waves, case.rec_cell[rm])
                n += 10
            t_all += time.perf_counter() - t0
            c = int(np.prod(case.shapes[d]))
            cells += c * n
            steps_done = n
        return {"workload": label, "gcells": round(cells / t_all / 1e9, 5), "seconds": round(t_all, 1),
                "sample_steps": steps_done}

    out = []
    c1 = configs.homogeneous_2d()
    fill_tables(c1)
    out.append(timed(c1, [0], "2D homogeneous 256x256 N=2"))
    c2 = configs.two_layer_2d()
    fill_tables(c2)
    out.append(timed(c2, [0], "2D two-layer 2048x2048 N=4 (first steps)"))
    c3 = configs.heterogeneous_3d(shape=(128, 128, 96), steps=2000, n_elem=16)
    fill_tables(c3)
    out.append(timed(c3, [0], "3D heterogeneous recipe on 128x128x96"))
    c4 = configs.batched_2d()
    configs.with_table(c4, *configs.random_relaxation_table(4000, c4.n_classes, c4.nmech))
    out.append(timed(c4, [0, 1, 2, 3], "batched 2D: 4 of the 64 shots"))
    c5 = configs.sweep_1d()
    _tables_or_random(c5, 3)
    out.append(timed(c5, list(range(0, 544, 68)), "1D sweep: 8 of the 544 domains"))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"oracle_timings": out, "cores": min(cores, os.cpu_count() or cores), "kind": "oracle FP64"}


def _time_steps(torch, sim, steps):
    """Milliseconds for `steps` full steps through fw_step (graph replay; the
    graph is captured before the timed region)."""
    sim.prepare()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _tune(sim):
    """Launch shape from the autotuner (timed live, no cache); results are
    bitwise independent of it.  The step graph is re-captured untimed."""
    from paper_2606_11103_amd.autotune import autotune
    cfg, _ = autotune(sim, steps=4, cache_path=None, use_cache=False)
    snap = sim.save_state()
    sim.step(32)
    sim.load_state(snap)
    return cfg


def bench_batched_launch(torch, steps=200, plane_kernels=None, plane_rows=None):
    """The 64-shot batched 2D launch alone, in the library's default launch
    shape (or with the given tile-kernel options): graph-replayed steps, then
    per-kernel HIP-event times, each against its algorithmic bytes (profiling
    the batched kernels in isolation)."""
    from paper_2606_11103_amd.native import FW_OPT_PLANE_KERNELS, FW_OPT_PLANE_ROWS
    from workloads import configs
    from workloads.adapters import to_simulation
    case = configs.batched_2d(steps=steps + 32)
    configs.with_table(case, *configs.random_relaxation_table(4000, case.n_classes, case.nmech))
    sim = to_simulation(case)
    if plane_kernels is not None:
        sim.set_option(FW_OPT_PLANE_KERNELS, plane_kernels)
    if plane_rows is not None:
        sim.set_option(FW_OPT_PLANE_ROWS, plane_rows)
    sim.step(32)                    # untimed: captures the step graph
    ms = _time_steps(torch, sim, steps) / steps
    sim.time_kernels(2)
    kern = sim.time_kernels(20)
    cells = case.cells()
    vb, pb, sb = algorithmic_bytes(case)
    frac = lambda b, t: round(b * cells / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return {"workload": case.name, "cells": cells, "steps": steps, "ms_per_step": round(ms, 4),
            "gcells": round(cells / ms / 1e6, 3), "bytes_per_cell": {"velocity": round(vb, 2), "pressure": round(pb, 2),
                                                                     "step": round(sb, 2)},
            "step_frac": frac(sb, ms), "velocity_ms": round(kern[0], 4), "velocity_frac": frac(vb, kern[0]),
            "pressure_ms": round(kern[1], 4), "pressure_frac": frac(pb, kern[1])}


def bench_batched(torch, steps=200):
    """64 ragged 2D shots (384^2..1536^2, N = 4, 4-layer media) advanced
    together in one tile list, vs the same shots run one at a time."""
    from workloads import configs
    from workloads.adapters import to_simulation
    case = configs.batched_2d(steps=steps + 32)
    configs.with_table(case, *configs.random_relaxation_table(4000, case.n_classes, case.nmech))
    sim = to_simulation(case)
    sim.step(32)                    # untimed: captures the step graph
    ms_default = _time_steps(torch, sim, steps)
    cfg = _tune(sim)
    ms = _time_steps(torch, sim, steps)
    batched = case.cells() * steps / (ms / 1e3) / 1e9
    del sim
    # plain: a sample of 8 shots, each its own simulation
    cells = 0
    tot = 0.0
    for s in range(0, 64, 8):
        one = configs.Case(**{**case.__dict__})
        one.shapes = [case.shapes[s]]
        one.class_maps = [case.class_maps[s]]
        one.class_base = [0]
        sl = slice(4 * s, 4 * s + 4)
        for f in ("c", "rho", "alpha0", "y", "b_over_a", "kappa", "d", "alpha"):
            setattr(one, f, getattr(case, f)[sl])
        one.src_domain = np.zeros(1, np.int32)
        one.src_cell = case.src_cell[s:s + 1]
        one.src_wave = case.src_wave[s:s + 1]
        rm = case.rec_domain == s
        one.rec_domain = np.zeros(int(rm.sum()), np.int32)
        one.rec_cell = case.rec_cell[rm]
        sim = to_simulation(one)
        sim.step(32)
        tot += _time_steps(torch, sim, steps)
        cells += one.cells()
        del sim
    plain = cells * steps / (tot / 1e3) / 1e9
    return {"workload": case.name, "cells": case.cells(), "steps": steps,
            "batched_gcells": round(batched, 3), "ms_per_step": round(ms / steps, 4),
            "step_frac": _step_frac(case, ms / steps),
            "launch_shape": cfg, "default_shape_gcells": round(case.cells() * steps / (ms_default / 1e3) / 1e9, 3),
            "plain_single_shot_gcells": round(plain, 3), "batched_vs_plain": round(batched / plain, 3),
            "plain_sample": "8 of the 64 shots, one simulation each"}


def _step_frac(case, ms_per_step):
    """Whole-step algorithmic bytes of the case over the step time, as a
    fraction of the 8 TB/s HBM peak."""
    return round(algorithmic_bytes(case)[2] * case.cells() / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)


def _tables_or_random(case, seed):
    """Cached calibrated tables of the case's classes, else (throughput only)
    a seeded random table of realistic strength."""
    from workloads import configs
    try:
        fill_tables(case, allow_fit=False)
        return "calibrated"
    except KeyError:
        configs.with_table(case, *configs.random_relaxation_table(seed, case.n_classes, case.nmech))
        return "random (calibration not cached)"


def bench_two_layer(torch, steps=400):
    """2D two-layer 2048 x 2048, N = 4, nonlinear, plane-wave line source."""
    from workloads import configs
    from workloads.adapters import to_simulation
    case = configs.two_layer_2d(steps=steps + 32)
    tab = _tables_or_random(case, 2)
    sim = to_simulation(case)
    sim.step(32)                    # untimed: captures the step graph
    ms = _time_steps(torch, sim, steps)
    # the same steps with the widened stencil (fourth order in time in every
    # direction): the 2D tile kernels' WIDE variants, tuned to the mean speed
    c_ref = float(np.mean(case.c))
    sim.set_widened_stencil(c_ref)
    sim.reset()
    sim.step(32)                    # untimed: re-captures the step graph
    ms_w = _time_steps(torch, sim, steps)
    return {"workload": case.name, "cells": case.cells(), "steps": steps, "tables": tab,
            "gcells": round(case.cells() * steps / (ms / 1e3) / 1e9, 3), "ms_per_step": round(ms / steps, 4),
            "step_frac": _step_frac(case, ms / steps),
            "widened_stencil": {"c_ref": round(c_ref, 1), "gcells": round(case.cells() * steps / (ms_w / 1e3) / 1e9, 3),
                                "ms_per_step": round(ms_w / steps, 4), "vs_taylor": round(ms_w / ms, 4)}}


def bench_paper_shape(torch, steps=100):
    """The 3D recipe at the grid of the paper's one timed run (499 x 499 x 1247
    cells, N = 2), for a like-for-like look at its derived 2.05e9
    cell-updates/s per H100 (context, not a target)."""
    from workloads import configs
    from workloads.adapters import to_simulation
    case = configs.heterogeneous_3d(shape=(499, 499, 1247), steps=steps + 32, n_elem=64, nmech=2)
    tab = _tables_or_random(case, 5)
    sim = to_simulation(case)
    sim.step(32)                    # untimed: captures the step graph
    ms_default = _time_steps(torch, sim, steps)
    cfg = _tune(sim)
    ms = _time_steps(torch, sim, steps)
    return {"workload": case.name, "cells": case.cells(), "steps": steps, "tables": tab,
            "gcells": round(case.cells() * steps / (ms / 1e3) / 1e9, 3), "ms_per_step": round(ms / steps, 4),
            "step_frac": _step_frac(case, ms / steps),
            "launch_shape": cfg, "default_shape_gcells": round(case.cells() * steps / (ms_default / 1e3) / 1e9, 3)}


def bench_sweep(torch, steps=2000):
    """1D sweep: 544 domains x 8192 cells, N = 2 and N = 4, one batched
    launch: the default resident step (each domain kept on chip by one
    workgroup), the whole 14800-step run with it, and the per-step kernels
    (FW_OPT_RESIDENT_1D 0) for comparison."""
    from paper_2606_11103_amd.native import FW_OPT_RESIDENT_1D
    from workloads import configs
    from workloads.adapters import to_simulation
    out = {}
    for nmech in (2, 4):
        case = configs.sweep_1d(nmech=nmech)
        tab = _tables_or_random(case, 3)
        sim = to_simulation(case)
        sim.step(32)                # untimed
        ms = _time_steps(torch, sim, steps)
        sim.reset()
        ms_full = _time_steps(torch, sim, case.n_steps)
        sim.set_option(FW_OPT_RESIDENT_1D, 0)
        sim.step(32)
        ms_ps = _time_steps(torch, sim, steps)
        del sim
        r = {"tables": tab, "gcells": round(case.cells() * steps / (ms / 1e3) / 1e9, 3),
             "ms_per_step": round(ms / steps, 5), "full_run_ms": round(ms_full, 2),
             "per_step_kernels_gcells": round(case.cells() * steps / (ms_ps / 1e3) / 1e9, 3)}
        if nmech == 2:
            out.update({"workload": case.name, "cells": case.cells(), "steps": steps,
                        "steps_of_full_run": case.n_steps, "step": "resident (one workgroup per domain)"})
            out.update(r)
        else:
            out["n4"] = r
    return out


def bench_adjoint(torch, steps=3000, ckpt=55):
    """Gradient of J = 1/2 dt sum (r - d)^2 w.r.t. c(x), alpha0(x) for the 16-shot
    1024^2 N = 4 workload over its 3000 steps (observed data: true model;
    current model: c x 0.99), forward with checkpoints every 55 steps +
    adjoint sweep (about 111 GB of checkpoints and segment states), vs the
    plain forward of the same steps."""
    from workloads import configs
    from workloads.adapters import to_simulation
    case = configs.adjoint_2d(steps=steps)
    fill_tables(case)
    true = to_simulation(case)
    true.step(steps)
    obs = true.read_receivers_device()
    del true
    case.c = case.c * 0.99
    sim = to_simulation(case)
    sim.set_class_alpha0(case.alpha0)
    sim.step(32)                    # untimed: captures the step graph
    sim.reset()
    ms_fwd = _time_steps(torch, sim, steps)
    sim.reset()
    work = sim.adjoint_workspace(steps, ckpt)
    work_bytes = work.numel()

    def gradient():
        sim.forward_checkpointed(steps, ckpt, work)
        tr = sim.read_receivers_device()
        res = case.dt * (tr - obs)
        gc, ga = sim.adjoint(steps, ckpt, work, res)
        return tr, gc, ga

    gradient()                      # untimed pass: first touch of the workspace
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    tr, gK, gs = gradient()
    e1.record()
    torch.cuda.synchronize()
    ms_grad = e0.elapsed_time(e1)
    misfit = float(0.5 * case.dt * ((tr.double() - obs.double()) ** 2).sum())
    finite = bool(torch.isfinite(gK).all() and torch.isfinite(gs).all())
    del work
    return {"workload": case.name + (" (%d steps)" % steps if steps == 3000 else " (%d of 3000 steps)" % steps),
            "cells": case.cells(), "steps": steps, "workspace_gb": round(work_bytes / 1e9, 1),
            "checkpoint_every": ckpt, "forward_ms": round(ms_fwd, 2), "gradient_ms": round(ms_grad, 2),
            "gradient_vs_forward": round(ms_grad / ms_fwd, 3),
            "forward_gcells": round(case.cells() * steps / (ms_fwd / 1e3) / 1e9, 3),
            "misfit": misfit, "gradients_finite": finite}


def bench_strength_map(torch, steps=100):
    """The benchmark workload with a per-voxel relaxation strength map (4 bytes
    per cell more for each update to read): Gcell-updates/s beside the plain
    run of the same case (the map's values do not change the traffic)."""
    from workloads.adapters import to_simulation
    case = bench_case()
    fill_tables(case)
    sim = to_simulation(case)
    sim.step(32)
    ms_plain = _time_steps(torch, sim, steps)
    sim.set_strength_map(torch.full((case.cells(),), 0.7, dtype=torch.float32, device="cuda"))
    sim.step(32)                    # untimed: re-captures the step graph
    ms_map = _time_steps(torch, sim, steps)
    cells = case.cells()
    return {"workload": case.name + " + strength map", "steps": steps,
            "gcells": round(cells * steps / (ms_map / 1e3) / 1e9, 3),
            "gcells_without_map": round(cells * steps / (ms_plain / 1e3) / 1e9, 3),
            "ms_per_step": round(ms_map / steps, 4), "ms_per_step_without_map": round(ms_plain / steps, 4),
            "extra_bytes_per_cell": 8}


def stream_probe(torch, reps=5, nmech=4):
    """Memory-traffic probes on the benchmark grid (fw_stream_probe): the
    velocity update's streams, the pressure update's, and a fused single
    pass, each as one flat sweep and as 64 x 4 tiles marching 48 planes."""
    from workloads.adapters import to_simulation
    case = bench_case(nmech=nmech)
    from workloads import configs
    configs.with_table(case, *configs.random_relaxation_table(1, case.n_classes, case.nmech))
    sim = to_simulation(case)
    cells = case.cells()
    N = case.nmech
    vel = 4 + 1 + 3 * 8 + 3 * 8 * N
    per_cell = {0: vel, 1: 3 * 4 + 8 + 1 + 8 * N, 2: (1 + 3 + 4 * N) * 8 + 1, 3: vel, 4: vel, 5: vel, 6: vel}
    out = {"workload": case.name + " (state streams only, no CPML)", "reps": reps}
    for mode, name in ((0, "velocity_streams"), (1, "pressure_streams"), (2, "fused_single_pass"),
                       (3, "velocity_streams_psi1_interleaved"), (4, "velocity_streams_psi1_v_interleaved"),
                       (5, "velocity_streams_psi1_blocked64"), (6, "velocity_streams_psi1_v_blocked64")):
        for order, oname in ((0, "flat"), (1, "marching_64x4x48")):
            ms = sim.stream_probe(mode, order, reps)
            out["%s_%s" % (name, oname)] = {"bytes_per_cell": per_cell[mode], "ms": round(ms, 3),
                                             "GBps": round(per_cell[mode] * cells / (ms / 1e3) / 1e9, 1)}
            print("# probe %s %s: %.3f ms" % (name, oname, ms), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def copy_probe(torch, gib, reps):
    """Plain copies of a known size (gib GiB read + gib GiB written per launch):
    the library's streaming copy kernel and torch's copy_.  Used to scale the
    FETCH_SIZE / WRITE_SIZE counters to bytes and as the practical bandwidth
    ceiling of the part."""
    import ctypes
    from paper_2606_11103_amd.native import check, lib
    n = int(gib * (1 << 30) // 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {"copy_probe_bytes_each_way": n * 4}
    for name in ("fw_device_copy", "torch_copy"):
        def run():
            if name == "fw_device_copy":
                check(lib.fw_device_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), n * 4,
                                         ctypes.c_void_p(stream.cuda_stream)))
            else:
                b.copy_(a)
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"avg_ms": round(ms, 4), "GBps_read_plus_write": round(2 * n * 4 / (ms / 1e3) / 1e9, 1)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--record", default=None,
                    help="append a JSONL record of the run (config hash, throughput, roofline, oracle, parity)")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--small", action="store_true", help="reduced grid for quick checks (not the benchmark)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, adjoint, two-layer 2D and 1D sweep workloads")
    ap.add_argument("--only", choices=("batched", "batched_launch", "adjoint", "two_layer", "sweep", "paper_shape",
                                       "strength_map"),
                    default=None,
                    help="run only one comparison workload and print its JSON (profiling)")
    ap.add_argument("--plane-kernels", type=int, default=None,
                    help="FW_OPT_PLANE_KERNELS for the headline run or --only batched_launch")
    ap.add_argument("--plane-rows", type=int, default=None,
                    help="FW_OPT_PLANE_ROWS for the headline run or --only batched_launch")
    ap.add_argument("--vel-planes", type=int, default=None, help="FW_OPT_VEL_PLANES for the headline run")
    ap.add_argument("--prs-planes", type=int, default=None, help="FW_OPT_PRS_PLANES for the headline run")
    ap.add_argument("--step-chunk", type=int, default=None,
                    help="FW_OPT_STEP_CHUNK for the headline run (0: whole-grid launches, -1: automatic)")
    ap.add_argument("--grid", type=int, nargs=3, default=None, metavar=("NX", "NY", "NZ"),
                    help="the benchmark recipe on another grid (profiling; not the benchmark line)")
    ap.add_argument("--nmech", type=int, default=4,
                    help="the benchmark recipe with another mechanism count (profiling; not the benchmark line)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--march-chunk", type=int, default=0)
    ap.add_argument("--rows-per-thread", type=int, default=0)
    ap.add_argument("--stream-probe", action="store_true",
                    help="only run the memory-traffic probes of the step's streams (fused-schedule bound)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (HBM counter calibration)")
    ap.add_argument("--adjoint-steps", type=int, default=3000,
                    help="steps of the adjoint workload (3000: the full workload; fewer for profiling)")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the FP64 oracle on bounded samples of each workload (host only)")
    args = ap.parse_args()
    if args.oracle_timings:
        print(json.dumps(oracle_timings()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe > 0:
        copy_probe(torch, args.copy_probe, max(args.steps, 1))
        return
    if args.stream_probe:
        torch.cuda.set_device(0)
        stream_probe(torch, nmech=args.nmech)
        return
    if args.only:
        torch.cuda.set_device(0)
        fn = dict(batched=bench_batched,
                  batched_launch=lambda t: bench_batched_launch(t, steps=args.steps, plane_kernels=args.plane_kernels,
                                                                plane_rows=args.plane_rows),
                  adjoint=lambda t: bench_adjoint(t, steps=args.adjoint_steps),
                  two_layer=bench_two_layer, sweep=bench_sweep, paper_shape=bench_paper_shape,
                  strength_map=bench_strength_map)[args.only]
        print(json.dumps(fn(torch)), flush=True)
        return
    from paper_2606_11103_amd.native import FW_OPT_MARCH_CHUNK, FW_OPT_ROWS_PER_THREAD, FW_OPT_TILE_ROWS
    from workloads.adapters import to_simulation

    torch.cuda.set_device(0)
    t0 = time.time()
    case = bench_case(full=not args.small, shape=args.grid, nmech=args.nmech)
    fill_tables(case)
    print("# workload %s built in %.1f s" % (case.name, time.time() - t0), file=sys.stderr, flush=True)
    sim = to_simulation(case)
    if args.rows_per_thread == 1:
        sim.set_option(FW_OPT_ROWS_PER_THREAD, 1)
    if args.tile_rows:
        sim.set_option(FW_OPT_TILE_ROWS, args.tile_rows)
    if args.rows_per_thread == 2:
        sim.set_option(FW_OPT_ROWS_PER_THREAD, 2)
    if args.march_chunk:
        sim.set_option(FW_OPT_MARCH_CHUNK, args.march_chunk)
    from paper_2606_11103_amd.native import (FW_OPT_PLANE_KERNELS, FW_OPT_PLANE_ROWS, FW_OPT_PRS_PLANES,
                                             FW_OPT_STEP_CHUNK, FW_OPT_VEL_PLANES)
    for key, val in ((FW_OPT_PLANE_KERNELS, args.plane_kernels), (FW_OPT_PLANE_ROWS, args.plane_rows),
                     (FW_OPT_VEL_PLANES, args.vel_planes), (FW_OPT_PRS_PLANES, args.prs_planes),
                     (FW_OPT_STEP_CHUNK, args.step_chunk)):
        if val is not None:
            sim.set_option(key, val)
    print("# simulation ready (%.1f GB workspace)" % (sim.workspace.numel() / 1e9), file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    sim.step(args.warmup)
    sim.prepare()                   # untimed: tile lists and the step graph's capture
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    # timed region: K full steps through fw_step (captured HIP graphs replayed
    # on torch's current stream), bracketed by HIP events on that stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    wall0 = time.perf_counter()
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    cells = case.cells()
    value = cells * args.steps / (ms_total / 1e3) / 1e9
    print("# timed %d graph-replayed steps: %.4f ms per step" % (args.steps, ms_step), file=sys.stderr, flush=True)

    # separate pass: the same steps launched eagerly with a HIP event pair
    # around every kernel, for the per-kernel figures (the state advances)
    kern_steps = max(5, min(args.steps, 50))
    kern_ms = sim.time_kernels(kern_steps)

    traces = sim.read_receivers()
    finite = bool(np.all(np.isfinite(traces[: min(case.n_steps, args.warmup + args.steps + kern_steps)])))

    b_vel, b_prs, b_step = algorithmic_bytes(case)
    ach_vel = b_vel * cells / (kern_ms[0] / 1e3) / 1e9
    ach_prs = b_prs * cells / (kern_ms[1] / 1e3) / 1e9
    ach_step = b_step * cells / (ms_step / 1e3) / 1e9
    chunk = step_chunk_planes(case, args.step_chunk, args.plane_kernels)
    n_vel_launches = 1 if chunk == 0 else -(-max(int(s[2]) for s in case.shapes) // chunk)
    meas = TRAFFIC_MEASURED.get((kernel_source_hash(), chunk))
    traffic = traffic_vel = None
    shape_opts = (args.tile_rows or args.rows_per_thread or args.march_chunk or
                  any(v is not None for v in (args.plane_kernels, args.plane_rows, args.vel_planes, args.prs_planes)))
    if meas is not None and not args.small and meas["workload"] == case.name and not (args.grid or args.nmech != 4) \
            and not shape_opts:
        traffic = round(meas["step_bytes"] / (ms_step / 1e3) / 1e9, 1)
        traffic_vel = round(meas["velocity_bytes"] / (kern_ms[0] / 1e3) / 1e9, 1)
    out = {
        "metric": "Gcell-updates/s (3D heterogeneous, %d mechanisms)" % case.nmech,
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name if not (args.small or args.grid or args.nmech != 4)
                   else case.name + " (not the benchmark)",
                   "cells": cells, "nmech": case.nmech, "pml_cells": case.pml_cells, "classes": case.n_classes,
                   "steps_of_full_run": case.n_steps, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "whole step (velocity + pressure + sources/receivers kernels, "
                                               "graph-replayed fw_step)",
                     "achieved": round(ach_step, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach_step / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_note": "FETCH_SIZE x 2 + WRITE_SIZE bytes of the step's kernels per step (L2 misses "
                                     "to the fabric: includes last-level-cache hits) / live step time, see profile",
                     "bytes_per_cell": round(b_step, 2), "avg_ms": round(ms_step, 4),
                     "step_schedule": ("whole-grid launches" if chunk == 0 else
                                       "interleaved velocity/pressure chunks of %d planes" % chunk),
                     "dominant_kernel": {"kernel": "velocity update", "achieved": round(ach_vel, 1),
                                         "frac": round(ach_vel / HBM_PEAK_GBS, 4), "traffic": traffic_vel,
                                         "bytes_per_cell": round(b_vel, 2), "avg_ms": round(kern_ms[0], 4),
                                         "launches_per_step": n_vel_launches,
                                         "avg_ms_per_launch": round(kern_ms[0] / n_vel_launches, 4)},
                     "pressure_kernel": {"achieved": round(ach_prs, 1), "frac": round(ach_prs / HBM_PEAK_GBS, 4),
                                         "bytes_per_cell": round(b_prs, 2), "avg_ms": round(kern_ms[1], 4)}},
        "kernels_ms": {"velocity": round(kern_ms[0], 4), "pressure": round(kern_ms[1], 4),
                       "sources_receivers": round(kern_ms[2], 4), "steps_timed": kern_steps},
        "traces_finite": finite,
        "wall_s": round(wall, 3),
    }
    if not args.no_extras and not args.small:
        del sim
        torch.cuda.empty_cache()
        print("# batched ...", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(torch)
        torch.cuda.empty_cache()
        print("# adjoint ...", file=sys.stderr, flush=True)
        out["adjoint"] = bench_adjoint(torch, steps=args.adjoint_steps)
        torch.cuda.empty_cache()
        print("# two-layer 2D ...", file=sys.stderr, flush=True)
        out["two_layer_2d"] = bench_two_layer(torch)
        torch.cuda.empty_cache()
        print("# 1D sweep ...", file=sys.stderr, flush=True)
        out["sweep_1d"] = bench_sweep(torch)
        torch.cuda.empty_cache()
        print("# paper's 3D shape, N = 2 ...", file=sys.stderr, flush=True)
        out["paper_shape_3d"] = bench_paper_shape(torch)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(gpu=True)
    print(json.dumps(out), flush=True)
    if args.record:
        with open(args.record, "a") as fh:
            fh.write(json.dumps(bench_record(out, kernel_source_hash())) + "\n")


if __name__ == "__main__":
    main()
