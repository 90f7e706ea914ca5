"""Pins of the oracle's closed forms against mathematics that does not reuse
the formula under test (Secs. 2.1, 2.2, 3.1, 3.3 of the paper)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import analytic, fdcoef
from oracle.solver import pml_profile, recursion_scale_derivatives, speed_noise, splitmix64


# ------------------------------------------------ staggered coefficients ----
def _stencil_apply_exact(coef, poly):
    """Staggered derivative at 0 with h = 1 of a polynomial given by its
    coefficient list, evaluated in exact rationals."""
    def f(x):
        return sum(Fraction(a) * x ** k for k, a in enumerate(poly))
    return sum(c * (f(Fraction(2 * m - 1, 2)) - f(Fraction(-(2 * m - 1), 2)))
               for m, c in enumerate(coef, start=1))


def test_fd_coefficients_exact_for_degree_le_7():
    coef = fdcoef.staggered_coefficients_exact(4)
    for deg in range(0, 8):
        poly = [0] * deg + [1]
        exact = 1 if deg == 1 else 0      # d/dx x^deg at 0
        assert _stencil_apply_exact(coef, poly) == exact, deg
    # order 8 exactly: x^9 is not differentiated exactly
    assert _stencil_apply_exact(coef, [0] * 9 + [1]) != 0


def test_fd_convergence_order_8():
    coef = fdcoef.staggered_coefficients(4)
    errs = []
    for h in (0.2, 0.1):
        x0 = 0.3
        approx = sum(c * (np.sin(x0 + (m - 0.5) * h) - np.sin(x0 - (m - 0.5) * h))
                     for m, c in enumerate(coef, start=1)) / h
        errs.append(abs(approx - np.cos(x0)))
    order = np.log2(errs[0] / errs[1])
    assert 7.6 < order < 8.4


def test_fd_coefficients_match_known_rational_values_independently():
    # consistency: the symbol K_d(k) of the operator equals k to O((k h)^8)
    coef = fdcoef.staggered_coefficients(4)
    k = np.array([1e-2, 2e-2])
    rel = np.abs(analytic.staggered_symbol(k, 1.0, coef).real - k) / k
    assert np.all(rel < 1e-14)


# ---------------------------------------- recursion coefficients (Sec 2.1) --
@pytest.mark.parametrize("kappa,d,alpha", [(1.0, 3e5, 2e7), (0.985, 1e6, 5e8), (0.99, 1e3, 1e5)])
def test_recursion_dc_gain_equals_continuous_gamma_at_zero(kappa, d, alpha):
    dt = 1e-8
    a, b = analytic.recursion_coefficients(kappa, d, alpha, dt)
    # sum of the impulse response a b^n = a/(1-b) must equal -gamma(0) of Eq. (gamma1)
    g0 = analytic.gamma(np.array([0.0]), kappa, [d], [alpha])[0]
    assert abs(a / (1.0 - b) + g0.real) <= 1e-13 * abs(g0)


@pytest.mark.parametrize("kappa,d,alpha", [(1.0, 3e5, 2e7), (0.985, 1e6, 5e8)])
def test_recursion_transfer_converges_to_gamma(kappa, d, alpha):
    # discrete transfer a/(1 - b e^{-i w dt}) -> -gamma(w) as dt -> 0 (first order)
    w = 2 * np.pi * np.array([1e6, 5e6, 2e7])
    g = analytic.gamma(w, kappa, [d], [alpha])
    errs = []
    for dt in (1e-10, 1e-11):
        a, b = analytic.recursion_coefficients(kappa, d, alpha, dt)
        errs.append(np.max(np.abs(a / (1 - b * np.exp(-1j * w * dt)) + g) / np.abs(g)))
    assert errs[1] < errs[0] / 5
    assert errs[1] < 1e-2


def test_scale_derivatives_by_finite_difference():
    kappa, d, alpha, dt = 0.99, 4e5, 3e7, 1.3e-8
    a_s, b_s = recursion_scale_derivatives(kappa, d, alpha, dt)
    h = 1e-6
    ap, bp = analytic.recursion_coefficients(kappa, d * (1 + h), alpha, dt)
    am, bm = analytic.recursion_coefficients(kappa, d * (1 - h), alpha, dt)
    assert abs((ap - am) / (2 * h) - a_s) < 1e-7 * abs(a_s)
    assert abs((bp - bm) / (2 * h) - b_s) < 1e-7 * abs(b_s)


# ----------------------------------------------- wavenumbers (Secs 2.2, 3.1) --
def test_kpred_without_relaxation_is_lossless_scaled():
    f = np.array([1e6, 7e6])
    k = analytic.k_pred(f, 1540.0, 0.99, 0.98, [0.0], [1e7], [0.0], [1e7])
    assert np.allclose(k, 2 * np.pi * f / 1540.0 * np.sqrt(0.99 * 0.98), rtol=1e-15)


def test_kpred_sign_convention_decays_and_is_causal():
    # a passive relaxation (d > 0) must attenuate: -Im k > 0, and add
    # dispersion with phase speed increasing with frequency
    f = np.logspace(6, np.log10(2e7), 16)
    args = (1540.0, 1.0, 1.0, [2e5, 1e6], [2e7, 2e8], [1e5, 3e5], [5e7, 1e9])
    a = analytic.model_attenuation(f, *args)
    c = analytic.model_phase_velocity(f, *args)
    assert np.all(a > 0)
    assert np.all(np.diff(c) > 0)


def test_kpred_matches_discrete_scheme_in_the_continuum_limit():
    # the exact wavenumber of the leapfrog/staggered scheme (with the discrete
    # memory-variable transfer) tends to Eq. (dispersion_relations)
    coef = fdcoef.staggered_coefficients(4)
    f = np.array([2e6, 8e6])
    w = 2 * np.pi * f
    c = 1540.0
    k1, k2 = 0.99, 0.995
    d1, a1 = np.array([2e5, 1e6]), np.array([2e7, 2e8])
    d2, a2 = np.array([1e5, 3e5]), np.array([5e7, 4e8])
    kc = analytic.k_pred(f, c, k1, k2, d1, a1, d2, a2)
    errs = []
    for dx in (2e-5, 2.5e-6):
        dt = 0.1 * dx / c
        A1, B1 = analytic.recursion_coefficients(k1, d1, a1, dt)
        A2, B2 = analytic.recursion_coefficients(k2, d2, a2, dt)
        S1 = analytic.discrete_stretch(w, k1, A1, B1, dt)
        S2 = analytic.discrete_stretch(w, k2, A2, B2, dt)
        kd = analytic.discrete_wavenumber(f, c, dx, dt, coef, S1, S2)
        errs.append(np.max(np.abs(np.conj(kd) - np.conj(kc)) / np.abs(kc)))
    assert errs[1] < errs[0] / 4
    assert errs[1] < 2e-3


@pytest.mark.parametrize("y", [0.4, 0.8, 1.3, 1.7])
def test_kk_relation_is_real_part_of_causal_power_law(y):
    # k(w) = w/c_inf - i a0 (i w)^y / cos(pi y / 2) is analytic in the lower
    # half plane (causal) with Im k = -a0 w^y; its real part over w must be
    # Eq. (kk_relation) up to the reference constant.
    alpha0, c0, f0 = 0.7, 1540.0, 1e6
    f = np.array([1e6, 3e6, 9e6, 2e7])
    w = 2 * np.pi * f
    a0 = analytic.alpha0_np_rad(alpha0, y)
    kc = -1j * a0 * (1j * w) ** y / np.cos(np.pi * y / 2)
    assert np.allclose(-kc.imag, analytic.power_law_alpha(f, alpha0, y), rtol=1e-12)
    inv_c = analytic.kk_inv_phase_velocity(f, c0, f0, alpha0, y)
    lhs = inv_c - inv_c[0]
    rhs = kc.real / w - kc.real[0] / w[0]
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-18)


def test_kk_relation_continuous_across_y_equal_one():
    f = np.array([2e6, 1.5e7])
    at1 = analytic.kk_inv_phase_velocity(f, 1540.0, 1e6, 0.5, 1.0)
    lo = analytic.kk_inv_phase_velocity(f, 1540.0, 1e6, 0.5, 1.0 - 1e-6)
    hi = analytic.kk_inv_phase_velocity(f, 1540.0, 1e6, 0.5, 1.0 + 1e-6)
    assert np.allclose(lo, at1, rtol=1e-9) and np.allclose(hi, at1, rtol=1e-9)
    assert np.all(np.diff(1 / at1) > 0)          # faster at higher frequency


def test_power_law_units():
    # 1 dB/(MHz cm) at 1 MHz is 100 dB/m = 100/8.6859 Np/m
    assert np.isclose(analytic.power_law_alpha(1e6, 1.0, 1.0), 100 / (20 / np.log(10)), rtol=1e-14)
    assert np.isclose(analytic.power_law_alpha(4e6, 0.5, 1.5), 0.5 * 8 * 100 / (20 / np.log(10)), rtol=1e-14)


def test_measurement_formulas():
    # a plane wave exp(-alpha x) over distance d: the two-receiver estimate is exact
    alpha, dist = 37.0, 0.01
    assert np.isclose(analytic.two_receiver_attenuation(1.0, np.exp(-alpha * dist), dist), alpha, rtol=1e-14)
    assert np.isclose(analytic.nrmse([1, 2, 3], [1, 2, 4]), np.sqrt(1 / 3) / 3, rtol=1e-14)
    assert np.isclose(analytic.reflection_db(1e-3, 1.0), -60.0)


# --------------------------------------------------- generators / profiles --
def test_splitmix64_published_reference_values():
    # first outputs of the reference splitmix64.c generator seeded with 0 and
    # 1234567 (the state advances by the golden gamma each call)
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        s0 = np.array([0, g, g * np.uint64(2)], dtype=np.uint64)
        out0 = splitmix64(s0)
    assert [int(x) for x in out0] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    with np.errstate(over="ignore"):
        s1 = np.array([1234567, np.uint64(1234567) + g], dtype=np.uint64)
        out1 = splitmix64(s1)
    assert [int(x) for x in out1] == [6457827717110365317, 3203168211198807973]


def test_speed_noise_range_and_mean():
    e = speed_noise(1 << 16, 0.01, 33)
    assert e.min() >= -0.01 and e.max() < 0.01
    assert abs(e.mean()) < 2e-4


def test_pml_profile_shape():
    n, P = 100, 20
    aF, bF = pml_profile(n, P, 1e-4, 1e-8, 1e-4, 1e6, 1540.0, True)
    aC, bC = pml_profile(n, P, 1e-4, 1e-8, 1e-4, 1e6, 1540.0, False)
    # interior untouched, both slabs active, a <= 0, 0 < b < 1
    assert np.all(aF[P:n - P] == 0) and np.all(aC[P:n - P] == 0)
    assert np.all(aC[:P] < 0) and np.all(aC[n - P:] < 0)
    assert np.all((bC[:P] > 0) & (bC[:P] < 1))
    # mirror symmetry of the cell profile about the centre of the grid
    assert np.allclose(aC, aC[::-1], rtol=1e-12)
    # faces: mirror of face i is face n-2-i (positions i+1/2 and n-3/2-i)
    assert np.allclose(aF[:n - 1], aF[:n - 1][::-1], rtol=1e-12)
