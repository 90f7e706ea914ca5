"""Host-side checks of bench.py: the algorithmic bytes behind the roofline
figures and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_algorithmic_bytes_of_the_benchmark():
    """3D, N = 4, 24-cell CPML on 960 x 960 x 720: slab fraction
    s = 2*24*(1/960 + 1/960 + 1/720) summed over axes; velocity
    4 + 1 + 24 + 96 + 8 s, pressure 12 + 8 + 32 + 1 + 8 s, whole step
    (1 + 3 + 4*4) * 8 + 1 + 16 s."""
    import bench
    from workloads import configs
    case = configs.heterogeneous_3d(shape=(960, 960, 720), steps=10, n_elem=4)
    vel, prs, step = bench.algorithmic_bytes(case)
    s = 48.0 / 960 + 48.0 / 960 + 48.0 / 720
    assert vel == pytest.approx(125 + 8 * s, rel=1e-12)
    assert prs == pytest.approx(53 + 8 * s, rel=1e-12)
    assert step == pytest.approx(161 + 16 * s, rel=1e-12)
    assert round(vel, 2) == 126.33 and round(step, 2) == 163.67


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_trace_errors_and_the_jsonl_record():
    """The parity figures of the record: relative L2 over all traces, the worst
    reached receiver (peak >= 1e-3 of the strongest), the count of those; and
    a record that carries them with a configuration hash that depends on the
    configuration only."""
    import json
    import numpy as np
    import bench
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((50, 4))
    ref[:, 3] *= 1e-6                         # below the reach: not counted
    got = ref.copy()
    got[:, 1] *= 1.01                         # one receiver 1 % off
    glob, worst, n = bench.trace_errors(got, ref)
    assert n == 3
    assert worst == pytest.approx(0.01, rel=1e-7)         # figures are rounded to 1e-10
    assert glob == pytest.approx(0.01 * np.linalg.norm(ref[:, 1]) / np.linalg.norm(ref), rel=1e-7)
    out = {"metric": "m", "value": 1.5, "unit": "u", "ms_per_step": 2.0,
           "config": {"workload": "w", "cells": 10},
           "roofline": {"frac": 0.6, "achieved": 4800.0, "traffic": 6000.0, "dominant_kernel": {"frac": 0.7}},
           "cpu_baseline": {"value": 0.1, "cores": 16, "parity": {"rel_l2": glob}}}
    r1 = bench.bench_record(out, "abc")
    r2 = bench.bench_record(dict(out, value=9.0), "abc")
    r3 = bench.bench_record(dict(out, config={"workload": "w", "cells": 11}), "abc")
    assert r1["config_hash"] == r2["config_hash"] != r3["config_hash"]
    assert r1["parity"]["rel_l2"] == glob and r1["oracle_cores"] == 16 and r1["roofline_frac"] == 0.6
    json.dumps(r1)


def test_step_chunk_planes_follows_the_automatic_rule():
    """The benchmark grid (960 x 960 x 720) and 384^3 run 120-plane chunks by
    default, the 256^3 grid and any 2D grid whole-grid launches; explicit
    values win."""
    import bench
    from types import SimpleNamespace as NS
    big = NS(ndim=3, shapes=[(960, 960, 720)])
    small = NS(ndim=3, shapes=[(256, 256, 256)])
    paper = NS(ndim=3, shapes=[(499, 499, 1247)])
    flat = NS(ndim=2, shapes=[(4096, 4096, 1)])
    mid = NS(ndim=3, shapes=[(384, 384, 384)])
    assert bench.step_chunk_planes(mid) == 120
    assert bench.step_chunk_planes(big) == 120
    assert bench.step_chunk_planes(paper) == 120
    assert bench.step_chunk_planes(small) == 0
    assert bench.step_chunk_planes(flat) == 0
    assert bench.step_chunk_planes(big, 0) == 0
    assert bench.step_chunk_planes(small, 16) == 16
    assert bench.step_chunk_planes(big, None, 0) == 0
    assert bench.step_chunk_planes(big, None, 1) == 120
