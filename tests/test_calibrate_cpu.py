"""Host side of the weight selection by simulated attenuation (no GPU):
spectra, two-receiver figures, measurement geometry and source spectrum."""
import math

import numpy as np

from oracle import analytic
from paper_2606_11103_amd import calibrate


def test_spectra_equal_fft_at_bin_frequencies():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((256, 3))
    dt = 1e-9
    f = np.fft.rfftfreq(256, dt)[[5, 17, 40]]
    P = calibrate.spectra(x, dt, f)
    ref = np.fft.rfft(x, axis=0)[[5, 17, 40]] * np.exp(-2j * np.pi * f * dt)[:, None]
    np.testing.assert_allclose(P, ref, rtol=1e-10, atol=1e-10)


def test_two_receiver_figures_invert_a_propagated_spectrum():
    """P_far = P_near exp(-alpha d - i w d / c) with the phase wrapped many
    times: alpha and c come back exactly (and agree with the oracle's
    intensity form of Sec. 4.1)."""
    for alpha, c, f, d in ((12.0, 1535.0, 3.7e6, 0.012), (250.0, 1560.0, 20e6, 0.0006), (0.5, 1540.0, 1e6, 0.0123)):
        Pn = 0.3 - 0.7j
        Pf = Pn * np.exp(-alpha * d - 1j * 2 * np.pi * f * d / c)
        a, cc = calibrate.two_receiver_figures(np.array([Pn]), np.array([Pf]), d, f, 1540.0)
        assert abs(a[0] - alpha) < 1e-9 * alpha
        assert abs(cc[0] - c) < 1e-9 * c
        assert abs(analytic.two_receiver_attenuation(Pn, Pf, d) - alpha) < 1e-9 * alpha


def test_errors_vanish_on_the_target_and_scale_with_offsets():
    f = calibrate.MEASURE_FREQS
    c0, a0, y = 1540.0, 0.5, 1.1
    at = analytic.power_law_alpha(f, a0, y)
    ct = 1.0 / analytic.kk_inv_phase_velocity(f, c0, 1e6, a0, y)
    nr, disp = calibrate.errors(at, ct, c0, a0, y)
    assert nr < 1e-12 and disp < 1e-9
    nr, disp = calibrate.errors(at + 0.01 * (at.max() - at.min()), ct + 2.0, c0, a0, y)
    assert abs(nr - 0.01) < 1e-12 and abs(disp - 2.0) < 1e-9


def test_measurement_geometry():
    dx = 1540.0 / (16 * 20e6)
    pairs = calibrate.measurement_cells(dx, 1540.0, 64)
    for k, f in enumerate(calibrate.MEASURE_FREQS):
        D = 10 * 1540.0 / f
        assert abs((pairs[k, 0] - 64) * dx - 0.05 * D) <= 0.5 * dx
        assert abs((pairs[k, 1] - 64) * dx - 0.8 * D) <= 0.5 * dx
    run = calibrate.SweepRun(np.ones((2, 2)), np.full((2, 2, 2), 1e6), np.full((2, 2, 2), 1e8))
    assert run.cells.max() < run.n_cells - run.pml
    # the pulse (5 sigma delay) has passed the farthest receiver by the last step
    far = (run.cells.max() - run.src_cell) * run.dx / run.c
    assert run.n_steps * run.dt > far + 10 / (2 * math.pi * 6e6)


def test_broadband_pulse_spectrum():
    """Spectral peak at 6 MHz and at least 2 % of the peak over 1-20 MHz."""
    dt = 1e-10
    w = calibrate.broadband_pulse(4000, dt).astype(np.float64)
    f = np.linspace(0.5e6, 25e6, 491)
    A = np.abs(calibrate.spectra(w[:, None], dt, f)[:, 0])
    assert abs(f[np.argmax(A)] - 6e6) <= 0.05e6
    band = (f >= 1e6) & (f <= 20e6)
    assert A[band].min() >= 0.02 * A.max()
