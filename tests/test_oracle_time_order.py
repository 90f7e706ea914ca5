"""Pins of the oracle's time-space-domain staggered coefficients (the
fourth-order-in-time operator of Sec. 3.3) against what the mathematics fixes:
the published two-point closed form, the Taylor limit r -> 0, the exact
one-cell-per-step transport at r = 1, and, through the stepping engine, the
continuous dispersion relation w = c k that the set is built to reproduce
(and which the Taylor set misses by its second-order time error)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import analytic, fdcoef
from oracle.solver import OracleSim


def _uniform_1d(n, dx, dt, c, fd_c_ref=None, rho=1000.0):
    return OracleSim(1, (n, 1, 1), dx, dt, 1, np.zeros(n, np.uint8), [c], [rho], [0.0],
                     [[1.0, 1.0]], np.zeros((1, 2, 1)), np.ones((1, 2, 1)), fd_c_ref=fd_c_ref)


def test_time_space_set_reduces_to_taylor_at_zero_courant():
    assert fdcoef.time_space_coefficients_exact(0.0, 4) == fdcoef.staggered_coefficients_exact(4)


@pytest.mark.parametrize("r", [0.1, 0.25, 0.5, 0.7, 0.9])
def test_two_point_set_matches_published_closed_form(r):
    # two-point time-space staggered operator: c1 = (9 - r^2) / 8,
    # c2 = (r^2 - 1) / 24 (Liu and Sen 2011, the M = 2 case)
    c1, c2 = fdcoef.time_space_coefficients_exact(r, 2)
    rr = Fraction(r) ** 2
    assert c1 == (9 - rr) / 8
    assert c2 == (rr - 1) / 24


def test_unit_courant_number_gives_the_two_point_difference():
    # at r = 1 the leapfrog step with the plain two-point difference is exact
    # in 1D, and every higher-order set must collapse onto it
    assert fdcoef.time_space_coefficients_exact(1.0, 4) == [1, 0, 0, 0]


def test_unit_courant_run_transports_a_pulse_one_cell_per_step():
    # d'Alembert at r = 1: a right-going pulse (p, v = p / (rho c)) moves one
    # cell per step without change of shape
    n, dx, c, rho = 600, 1e-4, 1500.0, 1000.0
    dt = dx / c
    sim = _uniform_1d(n, dx, dt, c, fd_c_ref=c, rho=rho)
    x = np.arange(n, dtype=np.float64)
    f = lambda s: np.exp(-0.5 * ((s - 150.0) / 6.0) ** 2)
    sim.p[:] = f(x)
    # v holds the half step before p's time level: v^{-1/2} at x + 1/2
    sim.v[0, :] = f(x + 0.5 + 0.5) / (rho * c)
    steps = 200
    sim.run(steps)
    assert np.max(np.abs(sim.p - f(x - steps))) < 1e-12


def _measured_rel_speed_error(coef_c_ref, r, f_lo, f_hi):
    dx, c = 1e-4, 1500.0
    dt = r * dx / c
    sim = _uniform_1d(9000, dx, dt, c, fd_c_ref=coef_c_ref)
    nt = 3400
    w = W.tone_burst(nt, dt, 1e6, 3).astype(np.float64)
    rec, _ = sim.run(nt, [2000], w[None, :], [2300, 2800])
    F = np.fft.rfft(rec, axis=0, n=8 * nt)
    f = np.fft.rfftfreq(8 * nt, dt)
    sel = (f > f_lo) & (f < f_hi)
    dist = 500 * dx
    coef = fdcoef.time_space_coefficients(r, 4) if coef_c_ref else fdcoef.staggered_coefficients(4)
    kth = analytic.discrete_wavenumber(f[sel], c, dx, dt, coef).real
    ph = -np.angle(F[sel, 1] / F[sel, 0])
    ph = ph + 2 * np.pi * np.round((kth * dist - ph) / (2 * np.pi))
    k_meas = ph / dist
    k_cont = 2 * np.pi * f[sel] / c
    return np.abs(k_meas - kth) / kth, np.abs(k_meas - k_cont) / k_cont


@pytest.mark.parametrize("r", [0.3, 0.6])
def test_time_space_run_follows_the_continuous_dispersion_relation(r):
    # the run follows the scheme's own discrete relation with either set ...
    own_ts, cont_ts = _measured_rel_speed_error(1500.0, r, 0.6e6, 1.3e6)
    own_ty, cont_ty = _measured_rel_speed_error(None, r, 0.6e6, 1.3e6)
    assert np.max(own_ts) < 1e-6 and np.max(own_ty) < 1e-6
    # ... and only the time-space set also matches w = c k (11.5 to 25 points
    # per wavelength: the Taylor set's second-order time error is
    # r^2 (k dx)^2 / 24 there, the time-space set's error is below 1e-6)
    assert np.max(cont_ts) < 2e-6
    assert np.min(cont_ty) > 1e-5
    assert np.max(cont_ty) > 50 * np.max(cont_ts)


def test_time_space_set_error_is_of_eighth_order():
    # closed-form check of the relation the set is built on: the mismatch of
    # sin(r b / 2) and r sum_m c_m sin((2m - 1) b / 2) shrinks by 2^9 when b
    # halves (leading term b^9), against 2^3 for the Taylor set at r > 0
    r = 0.5
    ts = np.array(fdcoef.time_space_coefficients(r, 4))
    ty = np.array(fdcoef.staggered_coefficients(4))
    odd = 2 * np.arange(1, 5) - 1

    def mismatch(coef, b):
        return abs(np.sin(r * b / 2) - r * np.sum(coef * np.sin(odd * b / 2)))

    b = 0.4
    assert mismatch(ts, b) / mismatch(ts, b / 2) == pytest.approx(2.0 ** 9, rel=0.05)
    assert mismatch(ty, b) / mismatch(ty, b / 2) == pytest.approx(2.0 ** 3, rel=0.05)


@pytest.mark.parametrize("ndim,shape", [(2, (48, 40, 1)), (3, (20, 18, 16))])
def test_energy_conserved_with_time_space_set(ndim, shape):
    # any fixed set keeps the divergence the negative transpose of the
    # gradient, so the discrete energy of a closed lossless box is conserved
    rng = np.random.default_rng(7)
    nx, ny, nz = shape
    cls = rng.integers(0, 3, (nz, ny, nx)).astype(np.uint8)
    dx, cmax = 1e-4, 1600.0
    dt = 0.4 * dx / cmax
    sim = OracleSim(ndim, shape, dx, dt, 1, cls, [1400, 1500, 1600], [900, 1000, 1100], [0.0] * 3,
                    np.ones((3, 2)), np.zeros((3, 2, 1)), np.ones((3, 2, 1)), fd_c_ref=1500.0)
    assert sim.fd != fdcoef.staggered_coefficients(4)
    nsrc = 80
    w = W.tone_burst(nsrc, dt, 1.5e6, 1, amplitude=1e3).astype(np.float64)
    nc = nx * ny * nz
    _, en = sim.run(600, [nc // 2 + 3], w[None, :], [0], energy=True)
    e = en[nsrc:]
    assert e[0] > 0
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-12
