"""Pins of the FP64 oracle solver against what the mathematics fixes:
exact discrete dispersion relations of the scheme, discrete energy
conservation, the CPML reflection bound, Fubini's small-distance harmonic
law, linearity, and the adjoint identities (dot product, finite differences)."""
import numpy as np
import pytest

import workloads as W
from oracle import analytic, fdcoef
from oracle.solver import OracleSim, misfit_gradient, recursion_coefficients

COEF = fdcoef.staggered_coefficients(4)


def _uniform_1d(n, dx, dt, c=1540.0, rho=1000.0, kappa=(1.0, 1.0), d=None, alpha=None,
                beta=0.0, pml=0, N=1):
    d = np.zeros((1, 2, N)) if d is None else np.asarray(d, dtype=float).reshape(1, 2, N)
    alpha = np.ones((1, 2, N)) if alpha is None else np.asarray(alpha, dtype=float).reshape(1, 2, N)
    return OracleSim(1, (n, 1, 1), dx, dt, N, np.zeros(n, np.uint8), [c], [rho], [beta],
                     [list(kappa)], d, alpha, pml_cells=pml)


def _spectra(rec, dt, pad=8):
    nt = rec.shape[0]
    F = np.fft.rfft(rec, axis=0, n=pad * nt)
    f = np.fft.rfftfreq(pad * nt, dt)
    return f, F


def test_lossless_plane_wave_matches_discrete_dispersion():
    dx, c = 1e-4, 1500.0
    dt = 0.4 * dx / c
    sim = _uniform_1d(8000, dx, dt, c=c)
    nt = 3000
    w = W.tone_burst(nt, dt, 1e6, 3).astype(np.float64)
    rec, _ = sim.run(nt, [2000], w[None, :], [2300, 2800])
    f, F = _spectra(rec, dt)
    sel = (f > 0.5e6) & (f < 1.6e6)
    dist = 500 * dx
    kth = analytic.discrete_wavenumber(f[sel], c, dx, dt, COEF).real
    ph = -np.angle(F[sel, 1] / F[sel, 0])
    ph = ph + 2 * np.pi * np.round((kth * dist - ph) / (2 * np.pi))
    assert np.max(np.abs(ph / dist - kth) / kth) < 1e-6
    # and the continuous speed differs measurably at this resolution
    assert np.max(np.abs(2 * np.pi * f[sel] / c - kth) / kth) > 1e-4


def test_relaxation_matches_discrete_complex_wavenumber():
    dx, c = 5e-5, 1540.0
    dt = 0.3 * dx / c
    kap = (0.995, 0.99)
    d = [[3e5, 1e6], [2e5, 5e5]]
    al = [[6e6, 6e7], [1e7, 1e8]]
    sim = _uniform_1d(8000, dx, dt, c=c, kappa=kap, d=d, alpha=al, N=2)
    nt = 4000
    w = W.tone_burst(nt, dt, 3e6, 2).astype(np.float64)
    rec, _ = sim.run(nt, [2000], w[None, :], [2300, 3000])
    f, F = _spectra(rec, dt)
    sel = (f > 1.5e6) & (f < 4.5e6)        # where the pulse spectrum is well above FP32 noise
    wv = 2 * np.pi * f[sel]
    S = []
    for i in range(2):
        a, b = recursion_coefficients(kap[i], np.array(d[i]), np.array(al[i]), dt)
        S.append(analytic.discrete_stretch(wv, kap[i], a, b, dt))
    kth = analytic.discrete_wavenumber(f[sel], c, dx, dt, COEF, S[0], S[1])
    dist = 700 * dx
    ph = -np.angle(F[sel, 1] / F[sel, 0])
    ph = ph + 2 * np.pi * np.round((kth.real * dist - ph) / (2 * np.pi))
    c_meas = wv / (ph / dist)
    c_th = wv / kth.real
    a_meas = analytic.two_receiver_attenuation(F[sel, 0], F[sel, 1], dist)
    assert np.max(np.abs(c_meas - c_th)) < 0.1                      # m/s
    assert np.max(np.abs(a_meas + kth.imag) / (-kth.imag)) < 5e-3    # 0.5 %


@pytest.mark.parametrize("ndim,shape", [(2, (48, 40, 1)), (3, (20, 18, 16))])
def test_energy_conserved_in_closed_lossless_box(ndim, shape):
    rng = np.random.default_rng(7)
    nx, ny, nz = shape
    cls = rng.integers(0, 3, (nz, ny, nx)).astype(np.uint8)
    dx, cmax = 1e-4, 1600.0
    dt = 0.4 * dx / cmax
    sim = OracleSim(ndim, shape, dx, dt, 1, cls, [1400, 1500, 1600], [900, 1000, 1100], [0.0] * 3,
                    np.ones((3, 2)), np.zeros((3, 2, 1)), np.ones((3, 2, 1)))
    nsrc = 80
    w = W.tone_burst(nsrc, dt, 1.5e6, 1, amplitude=1e3).astype(np.float64)
    nc = nx * ny * nz
    _, en = sim.run(600, [nc // 2 + 3], w[None, :], [0], energy=True)
    e = en[nsrc:]
    assert e[0] > 0
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-12


# A strongly attenuating tissue table (N = 4, fitted to alpha0 = 0.85
# dB/(MHz^y cm), y = 1.53): its gradient stretch has 1/kappa_1 - gamma_1(0)
# = 0.966 < 1, i.e. a low-frequency stretch below that of the lossless
# medium.  A CPML term merely added beside the tissue terms would drive the
# low-frequency stretch negative deep in the layer (gamma_pml(0) -> 1 where
# the CFS alpha vanishes) and the run would grow without bound; the layer
# stretching the lossy medium's own coordinate (product of the two stretches)
# stays passive.
STRONG_TISSUE = dict(
    kappa=(0.980001379052793, 0.9800003030837323),
    d=[[11132276.042165138, 4950831.385480297, 105869.96096906101, 2097849.1850146195],
       [300271.10171943426, 361055.74535571825, 63894.66504510635, 42995.96317345838]],
    alpha=[[2.9775631870261121e+08, 3.0412093520509440e+08, 3.0614357771185040e+08, 1.9911705816870743e+11],
           [4.5206743524231941e+07, 3.0048512686305606e+08, 4.5727538379535474e+07, 9.2388910540797506e+06]],
    N=4)
LOSSLESS = dict()


@pytest.mark.parametrize("medium,bar", [(LOSSLESS, -60.0), (STRONG_TISSUE, -60.0)], ids=["lossless", "tissue"])
def test_cpml_reflection_1d(medium, bar):
    """Plane wave at 16 points per wavelength onto a 20-cell CPML: the
    reflection (Sec. 4.3 definition) is measured against a run whose right end
    is out of reach, in a window that closes before the left end's echo."""
    c, f0 = 1540.0, 1e6
    dx = c / f0 / 16
    dt = 0.3 * dx / c
    nt = 1650

    def run(n, pml):
        sim = _uniform_1d(n, dx, dt, c=c, pml=pml, **medium)
        w = W.tone_burst(nt, dt, f0, 3).astype(np.float64)
        rec, _ = sim.run(nt, [200], w[None, :], [300])
        return rec[:, 0]

    ref = run(4000, 20)
    R = analytic.reflection_db(np.abs(run(400, 20) - ref).max(), np.abs(ref).max())
    assert R < bar
    # without the absorbing layer the end of the grid reflects (nearly) fully
    ref0 = run(4000, 0)
    R0 = analytic.reflection_db(np.abs(run(400, 0) - ref0).max(), np.abs(ref0).max())
    assert R0 > -3.0


MILD_TISSUE = dict(kappa=(0.99, 0.995), d=[[2e5], [1e5]], alpha=[[3e7], [5e7]])


@pytest.mark.parametrize("medium", [MILD_TISSUE, STRONG_TISSUE], ids=["mild", "strong"])
def test_cpml_long_run_no_growth(medium):
    c, f0 = 1540.0, 1e6
    dx = c / f0 / 16
    dt = 0.4 * dx / c
    sim = _uniform_1d(200, dx, dt, c=c, pml=20, **medium)
    w = W.tone_burst(400, dt, f0, 3).astype(np.float64)
    rec, _ = sim.run(20000, [100], w[None, :], [100])
    peak = np.abs(rec[:800]).max()
    assert np.abs(rec[-2000:]).max() < 1e-6 * peak


def test_nonlinear_second_harmonic_follows_fubini():
    c, rho, f0, beta = 1500.0, 1000.0, 1e6, 3.5
    dx = c / f0 / 32
    dt = 0.3 * dx / c
    n, nt = 4000, 11000
    xs = (400, 1000)
    from scipy.signal import hilbert

    sim = _uniform_1d(n, dx, dt, c=c, rho=rho, beta=beta, pml=20)
    w = W.tone_burst(nt, dt, f0, 12, amplitude=2e5).astype(np.float64)
    rec, _ = sim.run(nt, [100], w[None, :], [100 + xs[0], 100 + xs[1]])
    f = np.fft.rfftfreq(nt, dt)

    def env(x, fc):
        X = np.fft.rfft(x, axis=0)
        X[(f < 0.6 * fc) | (f > 1.4 * fc)] = 0
        return np.abs(hilbert(np.fft.irfft(X, n=nt, axis=0), axis=0))

    e1, e2 = env(rec, f0), env(rec, 2 * f0)
    for j, x in enumerate(xs):
        k = np.argmax(e1[:, j])
        p1, p2 = e1[k, j], e2[k, j]
        sigma = beta * 2 * np.pi * f0 * p1 * x * dx / (rho * c ** 3)   # x / shock distance
        assert sigma < 0.2
        assert abs(p2 / (sigma / 2 * p1) - 1.0) < 0.01


def test_linear_medium_scales_exactly():
    rng = np.random.default_rng(3)
    n = 40
    cls = rng.integers(0, 2, (n, n)).astype(np.uint8)
    dx = 1e-4
    dt = 0.3 * dx / 1600

    def run(scale):
        sim = OracleSim(2, (n, n, 1), dx, dt, 2, cls, [1500, 1600], [1000, 1050], [0.0, 0.0],
                        [[0.99, 0.995], [1.0, 0.98]], 10 ** rng.uniform(4, 6, (2, 2, 2)) * 0 + 3e5,
                        np.full((2, 2, 2), 5e7), pml_cells=6)
        w = W.tone_burst(200, dt, 2e6, 2).astype(np.float64) * scale
        rec, _ = sim.run(200, [n * n // 2], w[None, :], [5 * n + 5, 30 * n + 20])
        return rec

    assert np.array_equal(run(2.0), 2.0 * run(1.0))


def _adj_sim(rng, n=24, N=2, **kw):
    cls = rng.integers(0, 3, (n, n)).astype(np.uint8)
    kap = np.array([[0.99, 0.995], [0.985, 1.0], [1.0, 0.99]])
    d = 10 ** rng.uniform(4, 6, (3, 2, N))
    al = 10 ** rng.uniform(6, 8, (3, 2, N))
    dx = 1e-4
    dt = 0.3 * dx / 1600

    def mk(**k2):
        return OracleSim(2, (n, n, 1), dx, dt, N, cls, [1450, 1540, 1600], [950, 1000, 1080],
                         [0.0] * 3, kap, d, al, pml_cells=5, **k2)
    return mk


def test_adjoint_step_dot_product():
    rng = np.random.default_rng(11)
    sim = _adj_sim(rng)()
    x = {k: rng.standard_normal(getattr(sim, k).shape) for k in sim.STATE_FIELDS}
    y = {k: rng.standard_normal(getattr(sim, k).shape) for k in sim.STATE_FIELDS}
    for k in sim.STATE_FIELDS:
        getattr(sim, k)[...] = x[k]
    sim.run(1)
    Ax = {k: getattr(sim, k).copy() for k in sim.STATE_FIELDS}
    for k in sim.STATE_FIELDS:
        getattr(sim, k)[...] = x[k]
    lam = {k: y[k].copy() for k in y}
    sim.adjoint_step(lam, np.zeros(sim.nc), np.zeros(sim.nc))
    lhs = sum(np.sum(Ax[k] * y[k]) for k in Ax)
    rhs = sum(np.sum(x[k] * lam[k]) for k in x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_gradients_match_central_differences():
    rng = np.random.default_rng(5)
    mk = _adj_sim(rng)
    sim = mk()
    n = 24
    nt = 120
    w = W.tone_burst(nt, sim.dt, 3e6, 2).astype(np.float64)[None, :]
    src = [12 * n + 12]
    rec_cells = [3 * n + 6, 3 * n + 18, 20 * n + 10]
    # observed data from a perturbed medium so that the misfit is generic
    obs_sim = mk()
    obs_sim.K[...] *= 1.0 + 0.01 * rng.standard_normal(obs_sim.nc)
    obs, _ = obs_sim.run(nt, src, w, rec_cells)
    J, gK, gs, _ = misfit_gradient(sim, nt, src, w, rec_cells, obs)

    def J_of(K=None, s=None):
        sm = mk(d_scale=s)
        if K is not None:
            sm.K[...] = K
        r, _ = sm.run(nt, src, w, rec_cells)
        return 0.5 * sm.dt * np.sum((r - obs) ** 2)

    h = 1e-4
    for probe in (10 * n + 9, 15 * n + 14, 7 * n + 17):
        K0 = sim.K.copy()
        Kp, Km = K0.copy(), K0.copy()
        Kp[probe] *= 1 + h
        Km[probe] *= 1 - h
        fd = (J_of(K=Kp) - J_of(K=Km)) / (2 * h * K0[probe])
        assert abs(gK[probe] - fd) <= 1e-6 * abs(fd)
        sp, sm_ = np.ones(sim.nc), np.ones(sim.nc)
        sp[probe], sm_[probe] = 1 + h, 1 - h
        fd = (J_of(s=sp) - J_of(s=sm_)) / (2 * h)
        assert abs(gs[probe] - fd) <= 1e-6 * abs(fd)


def test_point_source_2d_follows_hankel_ratio():
    """2D homogeneous attenuating medium (the 256 x 256 homogeneous case):
    the spectral ratio between two receivers on a grid axis equals
    H0^(2)(k r2) / H0^(2)(k r1) with k the scheme's complex wavenumber."""
    from scipy.special import hankel2
    n, dx, c = 256, 5e-5, 1540.0
    dt = 0.4 * dx / c
    kap = (0.995, 0.99)
    d = np.array([[2e5, 8e5], [1e5, 4e5]])
    al = np.array([[2e7, 2e8], [3e7, 3e8]])
    sim = OracleSim(2, (n, n, 1), dx, dt, 2, np.zeros((n, n), np.uint8), [c], [1000.0], [0.0],
                    [list(kap)], d[None], al[None], pml_cells=20)
    nt = 600
    w = W.tone_burst(nt, dt, 3e6, 3).astype(np.float64)
    src = 128 * n + 128
    rec, _ = sim.run(nt, [src], w[None, :], [128 * n + 148, 128 * n + 208])
    f, F = _spectra(rec, dt)
    sel = (f > 2e6) & (f < 4e6)
    wv = 2 * np.pi * f[sel]
    S = []
    for i in range(2):
        a, b = recursion_coefficients(kap[i], d[i], al[i], dt)
        S.append(analytic.discrete_stretch(wv, kap[i], a, b, dt))
    k = analytic.discrete_wavenumber(f[sel], c, dx, dt, COEF, S[0], S[1])
    # numpy's forward FFT (kernel e^{-iwt}) gives the e^{+iwt} coefficients
    ratio = F[sel, 1] / F[sel, 0]
    pred = hankel2(0, k * 80 * dx) / hankel2(0, k * 20 * dx)
    assert np.max(np.abs(ratio - pred) / np.abs(pred)) < 0.02
