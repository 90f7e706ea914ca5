"""The C engine of the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU, no GPU).

Every parity claim rests on the oracle, so its engine is built with
-fsanitize=address,undefined and the oracle's own pins plus a small set of
parity inputs (1D/2D/3D, ragged shapes, N = 1..4, CPML, speed perturbation,
nonlinearity, the adjoint) run on that build in a child process (the
sanitizer runtime has to be loaded before the interpreter starts).  Any
out-of-bounds access, use of freed memory or undefined operation aborts the
child with a report."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENGINE_SRC = os.path.join(ROOT, "oracle", "fdtd_oracle.c")

PARITY_INPUTS = r"""
import numpy as np
from workloads import configs
from workloads.adapters import oracle_traces, to_oracle
from oracle.solver import misfit_gradient
cases = [configs.random_small(1, [(150, 1, 1), (97, 1, 1)], 1, 2, seed=1, steps=60, pml=6),
         configs.random_small(2, [(40, 33, 1), (29, 41, 1)], 3, 3, seed=2, steps=50, pml=5, nonlinear=True, noise=0.01),
         configs.random_small(3, [(21, 18, 17), (19, 23, 16)], 4, 3, seed=3, steps=30, pml=4, nonlinear=True, noise=0.01),
         configs.random_small(3, [(22, 20, 18)], 2, 2, seed=4, steps=30, pml=0)]
for c in cases:
    configs.with_table(c, *configs.random_relaxation_table(7, c.n_classes, c.nmech))
    r = oracle_traces(c)
    assert np.all(np.isfinite(r)) and np.abs(r).max() > 0
c = configs.random_small(2, [(30, 28, 1)], 2, 3, seed=5, steps=40, pml=4, nonlinear=False, noise=0.01, n_rec=4)
configs.with_table(c, *configs.random_relaxation_table(9, c.n_classes, c.nmech))
sim = to_oracle(c, 0)
obs = np.zeros((c.n_steps, len(c.rec_cell)))
J, gK, gs, _ = misfit_gradient(sim, c.n_steps, c.src_cell, c.waves.astype(np.float64)[c.src_wave],
                               c.rec_cell, obs)
assert np.all(np.isfinite(gK)) and np.all(np.isfinite(gs)) and J > 0
print("parity inputs done")
"""


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def sanitized_engine(tmp_path_factory):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path_factory.mktemp("asan") / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared",
                           "-fPIC", ENGINE_SRC, "-o", so, "-lm"])
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, ORACLE_ENGINE=so, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + HERE)
    return env


def _check(proc):
    text = proc.stdout + proc.stderr
    assert "AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]
    assert proc.returncode == 0, text[-4000:]


def test_oracle_pins_under_sanitizers(sanitized_engine):
    proc = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                           os.path.join(HERE, "test_oracle_solver.py"),
                           os.path.join(HERE, "test_oracle_crop.py"),
                           os.path.join(HERE, "test_oracle_interface.py"),
                           os.path.join(HERE, "test_oracle_time_order.py"),
                           "-k", "not 3d_interface_normal_to_z and not planted"],
                          cwd=ROOT, env=sanitized_engine, capture_output=True, text=True, timeout=900)
    _check(proc)


def test_parity_inputs_under_sanitizers(sanitized_engine):
    proc = subprocess.run([sys.executable, "-c", PARITY_INPUTS], cwd=ROOT, env=sanitized_engine,
                          capture_output=True, text=True, timeout=600)
    _check(proc)
    assert "parity inputs done" in proc.stdout
