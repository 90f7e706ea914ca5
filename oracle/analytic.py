"""Closed forms of the multiple-relaxation model, written out in FP64 (numpy).

Test infrastructure (the oracle): only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import anything under
``oracle/``.  Nothing here is shared with the product path.

Conventions (one reading, applied on both sides of every comparison):

* Time dependence e^{+i w t}.  The relaxation recursion of Sec. 2.1,
  Eq. (relaxation_psi), realises the stretch 1/s = 1/kappa - gamma with gamma of
  Eq. (gamma1) written with "+ i w"; with that sign the wavenumber of
  Eq. (dispersion_relations) has Im k < 0 for a decaying wave, so the
  attenuation is alpha = -Im k and the phase speed is w / Re k.
* alpha0 is given in dB/(MHz^y cm) as in the paper (Sec. 3.1); it is converted
  to Np/m with 20*log10(e) dB per neper and 100 cm per metre.
"""
import numpy as np

DB_PER_NEPER = 20.0 / np.log(10.0)


# ---------------------------------------------------------------- Sec. 3.1 --
def power_law_alpha(f_hz, alpha0_db, y):
    """Power-law attenuation alpha(f) = alpha0 f^y (Sec. 3.1,
    Eq. power_law_attenuation), f in MHz inside the law, result in Np/m."""
    f_mhz = np.asarray(f_hz, dtype=np.float64) / 1e6
    return alpha0_db * f_mhz ** y * 100.0 / DB_PER_NEPER


def alpha0_np_rad(alpha0_db, y):
    """alpha0 expressed in Np/m per (rad/s)^y, so that alpha(w) = a0 * w^y."""
    return alpha0_db * 100.0 / DB_PER_NEPER / (2.0 * np.pi * 1e6) ** y


def kk_inv_phase_velocity(f_hz, c0, f0_hz, alpha0_db, y):
    """1/c(w) from the Kramers-Kronig relation of Sec. 3.1 (Eq. kk_relation):
    1/c(w) = 1/c0 + a0 tan(pi y/2) (w^(y-1) - w0^(y-1)), y != 1.
    The paper excludes y = 1; there the limit of the same expression,
    1/c0 - (2/pi) a0 ln(w/w0), is used (one reading, see the tests for
    continuity across y = 1)."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    w0 = 2.0 * np.pi * f0_hz
    a0 = alpha0_np_rad(alpha0_db, y)
    if abs(y - 1.0) < 1e-12:
        return 1.0 / c0 - (2.0 / np.pi) * a0 * np.log(w / w0)
    return 1.0 / c0 + a0 * np.tan(np.pi * y / 2.0) * (w ** (y - 1.0) - w0 ** (y - 1.0))


def k_ground_truth(f_hz, c0, f0_hz, alpha0_db, y):
    """k_GT(w) = w / c(w) + i alpha(w) (Sec. 3.2)."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    return w * kk_inv_phase_velocity(f_hz, c0, f0_hz, alpha0_db, y) + 1j * power_law_alpha(f_hz, alpha0_db, y)


# ---------------------------------------------------------------- Sec. 2.2 --
def gamma(w, kappa, d, alpha):
    """gamma_i(w) = sum_nu (d/kappa^2) / (d/kappa + alpha + i w)  (Eq. gamma1)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.zeros(w.shape, dtype=np.complex128)
    for dn, an in zip(np.atleast_1d(d), np.atleast_1d(alpha)):
        g = g + (dn / kappa ** 2) / (dn / kappa + an + 1j * w)
    return g


def k_pred(f_hz, c, kappa1, kappa2, d1, alpha1, d2, alpha2):
    """Complex wavenumber of the multiple-relaxation model, Eq.
    (dispersion_relations):  k = (w/c) (1/(k1 k2) - g1/k2 - g2/k1 + g1 g2)^(-1/2)."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    g1 = gamma(w, kappa1, d1, alpha1)
    g2 = gamma(w, kappa2, d2, alpha2)
    inner = 1.0 / (kappa1 * kappa2) - g1 / kappa2 - g2 / kappa1 + g1 * g2
    return (w / c) * inner ** (-0.5)


def model_attenuation(f_hz, c, kappa1, kappa2, d1, alpha1, d2, alpha2):
    """alpha(f) = -Im k_pred (Np/m) under the e^{+iwt} convention."""
    return -np.imag(k_pred(f_hz, c, kappa1, kappa2, d1, alpha1, d2, alpha2))


def model_phase_velocity(f_hz, c, kappa1, kappa2, d1, alpha1, d2, alpha2):
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    return w / np.real(k_pred(f_hz, c, kappa1, kappa2, d1, alpha1, d2, alpha2))


# ------------------------------------------------ Sec. 2.1 recursion (FP64) --
def recursion_coefficients(kappa, d, alpha, dt):
    """Per-step coefficients of Eq. (relaxation_a) and Eq. (relaxation_b):
    b = exp(-(d/kappa + alpha) dt),  a = d / (kappa (d + kappa alpha)) (b - 1)."""
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    b = np.exp(-(d / kappa + alpha) * dt)
    a = d / (kappa * (d + kappa * alpha)) * (b - 1.0)
    return a, b


def discrete_stretch(w, kappa, a, b, dt):
    """Frequency response of the discrete stretched derivative: with the memory
    variable updated from the derivative of the same sub-step ("update, then
    use"), psi = a D / (1 - b e^{-i w dt}), so the operator multiplies D by
    S(w) = 1/kappa + sum_nu a_nu / (1 - b_nu e^{-i w dt})."""
    w = np.asarray(w, dtype=np.float64)
    S = np.full(w.shape, 1.0 / kappa, dtype=np.complex128)
    for an, bn in zip(np.atleast_1d(a), np.atleast_1d(b)):
        S = S + an / (1.0 - bn * np.exp(-1j * w * dt))
    return S


def staggered_symbol(k, dx, coef):
    """K_d(k) = (2/dx) sum_m c_m sin((2m-1) k dx / 2): the symbol of the
    staggered first derivative on e^{-ikx} is -i K_d(k)."""
    k = np.asarray(k, dtype=np.complex128)
    out = np.zeros(k.shape, dtype=np.complex128)
    for m, cm in enumerate(coef, start=1):
        out = out + cm * np.sin((2 * m - 1) * k * dx / 2.0)
    return 2.0 / dx * out


def staggered_symbol_dk(k, dx, coef):
    k = np.asarray(k, dtype=np.complex128)
    out = np.zeros(k.shape, dtype=np.complex128)
    for m, cm in enumerate(coef, start=1):
        out = out + cm * (2 * m - 1) * np.cos((2 * m - 1) * k * dx / 2.0)
    return out


def discrete_wavenumber(f_hz, c, dx, dt, coef, S1=None, S2=None):
    """Exact complex wavenumber of the 1D leapfrog staggered scheme:
    K_d(k) = 2 sin(w dt/2) / (c dt sqrt(S1 S2)), solved for k by Newton's method
    from the continuous k.  S1 = S2 = 1 gives the lossless scheme."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    S1 = np.ones_like(w, dtype=np.complex128) if S1 is None else np.asarray(S1)
    S2 = np.ones_like(w, dtype=np.complex128) if S2 is None else np.asarray(S2)
    rhs = 2.0 * np.sin(w * dt / 2.0) / (c * dt) / np.sqrt(S1 * S2)
    k = w / c / np.sqrt(S1 * S2)
    for _ in range(60):
        f = staggered_symbol(k, dx, coef) - rhs
        k = k - f / staggered_symbol_dk(k, dx, coef)
    return k


# ----------------------------------------------------- Sec. 4 measurements --
def two_receiver_attenuation(P_ref, P_att, dist):
    """Sec. 4.1: alpha = -(1/(2d)) ln(I_att / I_ref) with I = |P|^2 (Np/m)."""
    I_ref = np.abs(P_ref) ** 2
    I_att = np.abs(P_att) ** 2
    return -np.log(I_att / I_ref) / (2.0 * dist)


def nrmse(measured, target):
    """Sec. 4.1: NRMSE = RMSE / (alpha_max - alpha_min) of the target."""
    measured = np.asarray(measured)
    target = np.asarray(target)
    rmse = np.sqrt(np.mean((measured - target) ** 2))
    return rmse / (target.max() - target.min())


def reflection_db(p_reflected, p_incident):
    """Sec. 4.3, Eq. (reflection_coefficient_pml): R = 20 log10(p_refl/p_inc)."""
    return 20.0 * np.log10(p_reflected / p_incident)
