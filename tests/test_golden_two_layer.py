"""Checks of the stored oracle traces of the 2D two-layer workload
(tests/golden/two_layer_2d_2048_oracle.npz, written by
make_two_layer_traces.py with the oracle alone), independent of the GPU:

* the inputs stored with the traces are the workload generator's;
* discrete causality: one step moves information at most 8 cells (two
  staggered stencils of 4), so a receiver r rows below the source row reads
  exactly zero for the first floor((r - 28) / 8) steps;
* plane-wave amplitude: a soft line source of amplitude A radiates
  A / (2 CFL) each way (the injected pressure splits into two travelling
  waves), reduced by the power-law attenuation over the 36 rows to the first
  receiver (Sec. 3.1 law, 5 MHz);
* speed: the envelope crosses the upper layer no slower than its 1580 m/s
  and at most 2 % faster (causal dispersion and the nonlinear speed-up).
"""
import os

import numpy as np

from workloads import configs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_layer_2d_2048_oracle.npz")


def _load():
    g = np.load(GOLDEN)
    return g, configs.two_layer_2d(steps=int(g["steps"]))


def test_stored_inputs_are_the_workload():
    g, case = _load()
    np.testing.assert_array_equal(g["c"], case.c)
    np.testing.assert_array_equal(g["rho"], case.rho)
    np.testing.assert_array_equal(g["rec_cell"], case.rec_cell)
    np.testing.assert_array_equal(g["src_cell"], case.src_cell)
    np.testing.assert_array_equal(g["wave"], case.waves[0])
    assert float(g["dx"]) == case.dx and float(g["dt"]) == case.dt
    assert g["traces"].shape == (int(g["steps"]), len(case.rec_cell))
    assert np.all(np.isfinite(g["traces"]))


def test_discrete_causality():
    g, case = _load()
    tr = g["traces"]
    rows = case.rec_cell // case.shapes[0][0]
    for k, r in enumerate(rows):
        quiet = (r - 28) // 8
        assert np.all(tr[:min(quiet, tr.shape[0]), k] == 0.0), k
    assert np.abs(tr[:, 0]).max() > 0


def test_plane_wave_amplitude_and_speed():
    from scipy.signal import hilbert
    from oracle import analytic
    g, case = _load()
    tr = g["traces"].astype(np.float64)
    env = np.abs(hilbert(tr, axis=0))
    rows = case.rec_cell // case.shapes[0][0]
    cfl = 1580.0 * case.dt / case.dx
    alpha = analytic.power_law_alpha(5e6, 0.9, 1.1)              # Np/m, upper layer
    expect = 0.8e6 / (2.0 * cfl) * np.exp(-alpha * (rows[0] - 28) * case.dx)
    assert abs(env[:, 0].max() / expect - 1.0) < 0.05
    # envelope peaks of two receivers in the upper layer
    k1, k2 = 0, int(np.nonzero(rows < 1000)[0].max())
    t1, t2 = np.argmax(env[:, k1]), np.argmax(env[:, k2])
    c_env = (rows[k2] - rows[k1]) * case.dx / ((t2 - t1) * case.dt)
    assert 1580.0 <= c_env <= 1580.0 * 1.02, c_env
