"""Pins of the oracle's per-voxel relaxation strength scale (CPU, no GPU).

A voxel's scale s multiplies the recursion coefficients a of both operators
(Sec. 2.1, Eq. relaxation_psi), keeping b.  The discrete stretch of an
operator then reads S(w) = 1/kappa + s sum_nu a_nu / (1 - b_nu e^{-i w dt}),
so a homogeneous medium with a uniform scale propagates with the scheme's
exact discrete complex wavenumber for those stretches, and a step in s is a
stretch step, whose reflection follows the owner-cell layering pinned for
the interface handling (gradient stretch switching half a cell after the
divergence stretch).  A set-up that scales one operator only fails both."""
import numpy as np

import workloads as W
from oracle import analytic, fdcoef
from oracle.solver import OracleSim, recursion_coefficients

COEF = fdcoef.staggered_coefficients(4)
C0, RHO0 = 1540.0, 1000.0
KAP = (0.995, 0.99)
DD = [[3e5, 1e6], [2e5, 5e5]]
AL = [[6e6, 6e7], [1e7, 1e8]]


def _stretches(wv, dt, s):
    out = []
    for i in range(2):
        a, b = recursion_coefficients(KAP[i], np.array(DD[i]), np.array(AL[i]), dt)
        out.append(analytic.discrete_stretch(wv, KAP[i], s * a, b, dt))
    return out


def _run_uniform(s, one_operator=False):
    dx = 5e-5
    dt = 0.3 * dx / C0
    n = 8000
    sim = OracleSim(1, (n, 1, 1), dx, dt, 2, np.zeros(n, np.uint8), [C0], [RHO0], [0.0], [list(KAP)],
                    np.array([DD]), np.array([AL]), a_scale=np.full(n, s))
    if one_operator:       # planted mistake: the gradient operator left unscaled
        sim.coef["a1"][...] = sim.coef["a1"] / s
    nt = 4000
    w = W.tone_burst(nt, dt, 3e6, 2).astype(np.float64)
    rec, _ = sim.run(nt, [2000], w[None, :], [2300, 3000])
    return rec, dx, dt


def _check_uniform(rec, dx, dt, s):
    F = np.fft.rfft(rec, axis=0, n=8 * rec.shape[0])
    f = np.fft.rfftfreq(8 * rec.shape[0], dt)
    sel = (f > 1.5e6) & (f < 4.5e6)
    wv = 2 * np.pi * f[sel]
    S1, S2 = _stretches(wv, dt, s)
    kth = analytic.discrete_wavenumber(f[sel], C0, dx, dt, COEF, S1, S2)
    dist = 700 * dx
    a_meas = analytic.two_receiver_attenuation(F[sel, 0], F[sel, 1], dist)
    ph = -np.angle(F[sel, 1] / F[sel, 0])
    ph = ph + 2 * np.pi * np.round((kth.real * dist - ph) / (2 * np.pi))
    c_err = np.max(np.abs(wv / (ph / dist) - wv / kth.real))
    return np.max(np.abs(a_meas + kth.imag) / (-kth.imag)), c_err


def test_uniform_strength_follows_the_scaled_discrete_wavenumber():
    for s in (1.0, 0.35):
        rec, dx, dt = _run_uniform(s)
        ea, ec = _check_uniform(rec, dx, dt, s)
        assert ea < 5e-3 and ec < 0.1, (s, ea, ec)
    # attenuation scales with the strength while it is small
    rec1, dx, dt = _run_uniform(1.0)
    rec2, _, _ = _run_uniform(0.35)
    assert np.abs(rec2[:, 1]).max() > np.abs(rec1[:, 1]).max()


def test_scaling_one_operator_only_breaks_the_pin():
    rec, dx, dt = _run_uniform(0.35, one_operator=True)
    ea, ec = _check_uniform(rec, dx, dt, 0.35)
    assert ea > 0.05 or ec > 1.0


def _layer_reflection(w, Za, Zl, kl, Zb, L):
    cs, sn = np.cos(kl * L), np.sin(kl * L)
    m00, m01, m10, m11 = cs, -1j * Zl * sn, -1j * sn / Zl, cs
    al = m00 / Zb - m10
    be = (m01 / Zb - m11) / Za
    return -(al + be) / (al - be)


def test_strength_step_reflection_follows_the_owner_cell_layering():
    """s = 1 in cells < I, s = 0.1 from cell I on: the reflection referred to
    the face between cells I - 1 and I against the half-cell layer of the
    gradient stretch, at 40 and 80 points per wavelength (second order)."""
    errs = []
    f0 = 1e6
    for ppw in (40, 80):
        dx = C0 / f0 / ppw
        dt = 0.4 * dx / C0
        sc = ppw // 40
        n = 3000 * sc
        I = n // 2
        src, r1 = I - 600 * sc, I - 300 * sc
        nt = int(round(1.9 * (I - src + 300 * sc) * dx / C0 / dt))
        w = W.tone_burst(nt, dt, f0, 3).astype(np.float64)
        recs = []
        for step in (True, False):
            s = np.ones(n)
            if step:
                s[I:] = 0.1
            sim = OracleSim(1, (n, 1, 1), dx, dt, 2, np.zeros(n, np.uint8), [C0], [RHO0], [0.0], [list(KAP)],
                            np.array([DD]), np.array([AL]), a_scale=s)
            r, _ = sim.run(nt, [src], w[None, :], [r1])
            recs.append(r[:, 0])
        F = np.fft.rfft(recs[0], n=8 * nt)
        H = np.fft.rfft(recs[1], n=8 * nt)
        f = np.fft.rfftfreq(8 * nt, dt)
        sel = (f > 0.6 * f0) & (f < 1.4 * f0)
        wv = 2 * np.pi * f[sel]
        S1a, S2a = _stretches(wv, dt, 1.0)
        S1b, S2b = _stretches(wv, dt, 0.1)
        k1 = analytic.discrete_wavenumber(f[sel], C0, dx, dt, COEF, S1a, S2a)
        xI, x1 = (I - 0.5) * dx, r1 * dx
        R = (F[sel] - H[sel]) / H[sel] * np.exp(1j * k1 * 2 * (xI - x1))
        Z = lambda S1, S2: RHO0 * C0 * np.sqrt(S2 / S1)
        pred = _layer_reflection(wv, Z(S1a, S2a), Z(S1a, S2b), wv / C0 / np.sqrt(S1a * S2b), Z(S1b, S2b),
                                 0.5 * dx)
        errs.append(np.max(np.abs(R - pred) / np.abs(pred)))
    assert errs[0] < 2e-2 and errs[1] < 6e-3, errs
    assert errs[0] / errs[1] > 3.0
