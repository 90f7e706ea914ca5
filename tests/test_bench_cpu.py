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
