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


def _exact_2d(n, h, c, rho, sigma, t_p, t_v):
    """Continuous solution of p_t = -rho c^2 div v, rho v_t = -grad p on the
    plane, from p(x, 0) = Gaussian, v(x, 0) = 0 (spectral, on a grid large
    enough that the field stays clear of its edges): p at cells at time t_p,
    v at the faces (x + h/2, y) and (x, y + h/2) at time t_v."""
    k = 2 * np.pi * np.fft.fftfreq(n, h)
    KX, KY = np.meshgrid(k, k, indexing="xy")
    kk = np.sqrt(KX ** 2 + KY ** 2)
    x = (np.arange(n) - n / 2) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    G = np.fft.fft2(np.exp(-(X ** 2 + Y ** 2) / (2 * sigma ** 2)))
    w = c * kk
    p = np.real(np.fft.ifft2(G * np.cos(w * t_p)))
    s = np.where(kk > 0, np.sin(w * t_v) / np.where(kk > 0, w, 1.0), t_v)
    vx = np.real(np.fft.ifft2(-1j * KX / rho * G * s * np.exp(1j * KX * h / 2)))
    vy = np.real(np.fft.ifft2(-1j * KY / rho * G * s * np.exp(1j * KY * h / 2)))
    return p, vx, vy


def _pulse_error_2d(n, r, fd_c_ref=None, off_axis=False, L=0.0128, c=1500.0, rho=1000.0):
    h = L / n
    dt = r * h / c
    sigma = L / 24
    steps = int(round(0.2 * L / c / dt))
    sim = OracleSim(2, (n, n, 1), h, dt, 1, np.zeros((1, n, n), np.uint8), [c], [rho], [0.0],
                    [[1.0, 1.0]], np.zeros((1, 2, 1)), np.ones((1, 2, 1)), fd_c_ref=fd_c_ref, off_axis=off_axis)
    p0, vx, vy = _exact_2d(n, h, c, rho, sigma, 0.0, -dt / 2)
    sim.p[:] = p0.reshape(-1)
    sim.v[0, :] = vx.reshape(-1)
    sim.v[1, :] = vy.reshape(-1)
    sim.run(steps)
    pe, _, _ = _exact_2d(n, h, c, rho, sigma, steps * dt, 0.0)
    return np.linalg.norm(sim.p - pe.reshape(-1)) / np.linalg.norm(pe)


def test_widened_stencil_coefficients_closed_forms():
    # b = r^2 / 24; the on-axis moments shift by 2 (d - 1) b, which moves c_1
    # alone (the shift solves the moment system with (1, 0, 0, 0)); no shift
    # and no b at r = 0 (the Taylor set)
    for ndim in (2, 3):
        c, b = fdcoef.isotropic_time_space_coefficients_exact(0.45, ndim, 4)
        ts = fdcoef.time_space_coefficients_exact(0.45, 4)
        assert b == Fraction(0.45) ** 2 / 24
        assert c[0] == ts[0] - 2 * (ndim - 1) * b and c[1:] == ts[1:]
        c0, b0 = fdcoef.isotropic_time_space_coefficients_exact(0.0, ndim, 4)
        assert b0 == 0 and c0 == fdcoef.staggered_coefficients_exact(4)


def test_widened_stencil_is_fourth_order_in_time_for_a_2d_pulse():
    # a Gaussian pulse (every propagation direction) against the continuous
    # solution, refined at fixed r = 0.5: the error falls 4x per halving with
    # the Taylor and the on-axis time-space sets (second order: their mixed
    # (k_x k_y)^2 terms), 16x with the widened stencil (fourth order)
    r = 0.5
    ty = [_pulse_error_2d(n, r) for n in (96, 192)]
    ts = [_pulse_error_2d(n, r, fd_c_ref=1500.0) for n in (96, 192)]
    iso = [_pulse_error_2d(n, r, fd_c_ref=1500.0, off_axis=True) for n in (96, 192)]
    assert 3.5 < ty[0] / ty[1] < 4.6
    assert 3.5 < ts[0] / ts[1] < 4.6
    assert iso[0] / iso[1] > 13.0
    assert iso[1] < ts[1] / 50


def test_energy_conserved_with_widened_stencil():
    # the divergence takes the same widened stencil, so it stays the negative
    # transpose of the gradient and a closed lossless heterogeneous box keeps
    # its discrete energy (2D and 3D)
    for ndim, shape in ((2, (48, 40, 1)), (3, (20, 18, 16))):
        rng = np.random.default_rng(9)
        nx, ny, nz = shape
        cls = rng.integers(0, 3, (nz, ny, nx)).astype(np.uint8)
        dx, cmax = 1e-4, 1600.0
        dt = 0.35 * dx / cmax
        sim = OracleSim(ndim, shape, dx, dt, 1, cls, [1400, 1500, 1600], [900, 1000, 1100], [0.0] * 3,
                        np.ones((3, 2)), np.zeros((3, 2, 1)), np.ones((3, 2, 1)), fd_c_ref=1500.0, off_axis=True)
        assert sim.fd_b > 0
        nsrc = 80
        w = W.tone_burst(nsrc, dt, 1.5e6, 1, amplitude=1e3).astype(np.float64)
        nc = nx * ny * nz
        _, en = sim.run(500, [nc // 2 + 3], w[None, :], [0], energy=True)
        e = en[nsrc:]
        assert e[0] > 0
        assert np.max(np.abs(e - e[0])) / e[0] < 1e-12
