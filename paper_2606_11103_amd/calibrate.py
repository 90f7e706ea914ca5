"""Choice of the objective weight w by simulated attenuation (Sec. 3.2).

The host fit (relax.fit_class) produces one parameter set per weight w of the
objective.  The paper keeps, for each (alpha0, y) class, the weight whose
*simulated* attenuation is closest to the power law.  Here every candidate
of every class becomes one domain of a single batched 1D run on the GPU
(the ragged-batch path of the step kernels), and the simulated attenuation
and phase speed are measured as in Sec. 4.1-4.2:

* plane wave from a broadband source (first derivative of a Gaussian with its
  spectral peak at 6 MHz) in a 1D domain with CPML at both ends;
* for each of the eight measurement frequencies f_k = 1 + 2.714 k MHz, two
  receivers at 0.05 D and 0.8 D from the source, D = 10 wavelengths at f_k;
* alpha(f_k) = ln|P_near / P_far| / distance and c(f_k) = 2 pi f_k distance /
  unwrapped phase delay, with P the discrete Fourier transform of the trace
  at exactly f_k;
* attenuation NRMSE against alpha0 f^y (RMSE over the eight frequencies
  divided by the target's range) and dispersion RMSE against the
  Kramers-Kronig phase speed of Eq. (kk_relation).

Selection (relax.choose with the simulated figures): the lowest simulated
NRMSE among the candidates within both bars of the failure label (10 % NRMSE,
5 m/s dispersion error), else among all; ties to the lower dispersion error,
then to the smaller w.
"""
import math

import numpy as np

from . import relax

MEASURE_FREQS = relax.MEASURE_FREQS


def measurement_cells(dx, c, src_cell, freqs=MEASURE_FREQS):
    """[n_freq][2] cells at 0.05 D and 0.8 D from the source, D = 10 c / f."""
    out = np.zeros((len(freqs), 2), dtype=np.int64)
    for k, f in enumerate(freqs):
        D = 10.0 * c / f
        out[k] = (src_cell + int(round(0.05 * D / dx)), src_cell + int(round(0.8 * D / dx)))
    return out


def broadband_pulse(n_t, dt, f_peak=6e6):
    """First derivative of a Gaussian, spectral peak at f_peak, centred at
    5 sigma, unit peak amplitude, sampled at t_s = (s + 1) dt (float32)."""
    sigma = 1.0 / (2.0 * math.pi * f_peak)
    t = (np.arange(n_t, dtype=np.float64) + 1.0) * dt
    u = (t - 5.0 * sigma) / sigma
    return (-u * np.exp(-0.5 * u * u) * math.exp(0.5)).astype(np.float32)


def spectra(traces, dt, freqs):
    """DFT of each column of traces [n_t][m] at the given frequencies, sample s
    at time (s + 1) dt, kernel e^{-i 2 pi f t}: [len(freqs)][m] complex."""
    t = (np.arange(traces.shape[0], dtype=np.float64) + 1.0) * dt
    E = np.exp(-2j * np.pi * np.outer(freqs, t))
    return E @ traces.astype(np.float64)


def two_receiver_figures(P_near, P_far, dist, f, c_guess):
    """(alpha in Np/m, phase speed in m/s) from the spectra at two receivers
    dist apart; the phase delay is unwrapped around the delay at c_guess."""
    alpha = np.log(np.abs(P_near) / np.abs(P_far)) / dist
    ph = -np.angle(P_far / P_near)
    kd = 2.0 * np.pi * f / c_guess * dist
    ph = ph + 2.0 * np.pi * np.round((kd - ph) / (2.0 * np.pi))
    return alpha, 2.0 * np.pi * f * dist / ph


def errors(alpha_sim, c_sim, c0, alpha0_db, y, freqs=MEASURE_FREQS):
    """(attenuation NRMSE, dispersion RMSE) of one domain's measurements."""
    kt = relax.target_wavenumber(freqs, c0, alpha0_db, y)
    at = kt.imag
    ct = 2.0 * np.pi * np.asarray(freqs) / kt.real
    nr = math.sqrt(np.mean((alpha_sim - at) ** 2)) / (at.max() - at.min())
    return nr, math.sqrt(np.mean((c_sim - ct) ** 2))


class SweepRun:
    """One batched 1D run: domain j holds relaxation table j (kappa [2],
    d [2][N], alpha [2][N], as fitted) at speed c and density rho.  With
    step_match the tables are relax.step_matched to the run's time step
    before they are simulated (self.kappa, self.d, self.alpha hold what runs)."""

    def __init__(self, kappa, d, alpha, c=1540.0, rho=1000.0, n_cells=8192, pml=24, src_cell=64, cfl=0.2,
                 f_top=20e6, ppw=16, step_match=True):
        self.c, self.rho = float(c), float(rho)
        self.dx = c / (ppw * f_top)
        self.dt = cfl * self.dx / c
        kappa = np.asarray(kappa, dtype=np.float64)
        d = np.asarray(d, dtype=np.float64)
        alpha = np.asarray(alpha, dtype=np.float64)
        if step_match:
            kappa, d, alpha = relax.step_matched(kappa, d, alpha, self.dt)
        self.kappa, self.d, self.alpha = kappa, d, alpha
        self.n_dom = self.kappa.shape[0]
        self.nmech = self.d.shape[2]
        self.n_cells, self.pml, self.src_cell = int(n_cells), int(pml), int(src_cell)
        self.pairs = measurement_cells(self.dx, c, src_cell)
        if self.pairs.max() >= n_cells - pml:
            raise ValueError("domain too short for the farthest receiver")
        self.cells = np.unique(self.pairs.ravel())
        self.n_steps = int(round((int(self.cells.max()) - src_cell) * self.dx / c / self.dt)) + 2000

    def run(self):
        """Simulate every domain; returns traces [n_steps][n_dom][n_cells_rec]."""
        from .sim import Simulation
        nd = self.n_dom
        sim = Simulation(1, [(self.n_cells, 1, 1)] * nd, self.dx, self.dt, self.nmech, self.pml)
        try:
            sim.set_media([np.zeros(self.n_cells, np.uint8)] * nd, np.arange(nd), np.full(nd, self.c),
                          np.full(nd, self.rho), np.zeros(nd))
            sim.set_relaxation_table(self.kappa, self.d, self.alpha)
            sim.set_sources(np.arange(nd), np.full(nd, self.src_cell), np.zeros(nd),
                            broadband_pulse(self.n_steps, self.dt)[None, :])
            m = self.cells.size
            sim.set_receivers(np.repeat(np.arange(nd), m), np.tile(self.cells, nd), self.n_steps)
            sim.step(self.n_steps)
            tr = sim.read_receivers()
        finally:
            sim.close()
        return tr.reshape(self.n_steps, nd, self.cells.size)

    def measure(self, traces, chunk=256):
        """(alpha [n_dom][n_freq], c [n_dom][n_freq]) from run()'s traces."""
        nf = len(MEASURE_FREQS)
        alpha = np.zeros((self.n_dom, nf))
        cph = np.zeros((self.n_dom, nf))
        col = {int(v): i for i, v in enumerate(self.cells)}
        for k, f in enumerate(MEASURE_FREQS):
            a, b = (col[int(v)] for v in self.pairs[k])
            dist = (self.pairs[k, 1] - self.pairs[k, 0]) * self.dx
            for s in range(0, self.n_dom, chunk):
                e = min(self.n_dom, s + chunk)
                P = spectra(np.concatenate([traces[:, s:e, a], traces[:, s:e, b]], axis=1), self.dt, [f])[0]
                alpha[s:e, k], cph[s:e, k] = two_receiver_figures(P[:e - s], P[e - s:], dist, f, self.c)
        return alpha, cph


def select_weights(fits, c=1540.0, rho=1000.0, **kw):
    """For fitted classes (relax.fit_class results carrying "cands"), simulate
    every candidate and pick the weight by relax.choose on the simulated
    figures.  Returns (chosen fits, nrmse [n_class][n_cand], disp [n_class][n_cand])."""
    n_cls = len(fits)
    n_cand = len(fits[0]["cands"])
    flat = [cd for ft in fits for cd in ft["cands"]]
    if any(len(ft["cands"]) != n_cand for ft in fits):
        raise ValueError("every class needs the same number of candidates")
    run = SweepRun([cd["kappa"] for cd in flat], [cd["d"] for cd in flat], [cd["alpha"] for cd in flat],
                   c=c, rho=rho, **kw)
    alpha, cph = run.measure(run.run())
    nr = np.zeros((n_cls, n_cand))
    dp = np.zeros((n_cls, n_cand))
    chosen = []
    for i, ft in enumerate(fits):
        for j in range(n_cand):
            nr[i, j], dp[i, j] = errors(alpha[i * n_cand + j], cph[i * n_cand + j], c, ft["alpha0"], ft["y"])
        j = relax.choose(ft["cands"], nr[i], dp[i])
        pick = dict(ft["cands"][j])
        pick.update(c=ft["c"], alpha0=ft["alpha0"], y=ft["y"], nmech=ft["nmech"], sim_nrmse=float(nr[i, j]),
                    sim_disp=float(dp[i, j]), failed=not relax.passes(nr[i, j], dp[i, j]))
        chosen.append(pick)
    return chosen, nr, dp


def tone_burst(n_t, dt, f0, n_cycles, amplitude=1.0):
    """Gaussian-modulated sine: A sin(2 pi f0 (t - t0)) exp(-((t - t0)/sigma)^2),
    sigma = n_cycles / (2 f0), t0 = 4 sigma, sampled at t_s = (s + 1) dt."""
    sigma = n_cycles / (2.0 * f0)
    t = (np.arange(n_t, dtype=np.float64) + 1.0) * dt - 4.0 * sigma
    return (amplitude * np.sin(2.0 * np.pi * f0 * t) * np.exp(-(t / sigma) ** 2)).astype(np.float32)


def pml_reflection(kappa, d, alpha, c=1540.0, rho=1000.0, f0=1e6, ppw=16, cfl=0.2, pml_wavelengths=3.0,
                   depth_wavelengths=5.0, n_cycles=3, step_match=True):
    """Reflection coefficient of the CPML for each relaxation table, in dB
    (Sec. 4 protocol, 1D plane wave): source below the top layer, a receiver
    at 0.8 D towards the bottom layer D = 5 wavelengths away, 1 MHz
    Gaussian-modulated pulse, layer thickness 3 wavelengths.  Each table runs
    in two domains of one batched launch: one that ends in the layer and one
    long enough that nothing returns from its far end within the window; the
    reflected wave is the difference of the two receiver traces,
    R = 20 log10(max|difference| / max|incident|).  With step_match the
    tables are relax.step_matched to the run's time step first."""
    from .sim import Simulation
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    n_tab, nmech = kappa.shape[0], d.shape[2]
    lam = c / f0
    dx = lam / ppw
    dt = cfl * dx / c
    if step_match:
        kappa, d, alpha = relax.step_matched(kappa, d, alpha, dt)
    P = int(round(pml_wavelengths * ppw))
    D = int(round(depth_wavelengths * ppw))
    src = P + 4
    rec = src + int(round(0.8 * D))
    sigma = n_cycles / (2.0 * f0)
    # the reflected pulse has passed the receiver (8 sigma long, centred at
    # 4 sigma after the travel time) by the end of the window
    travel = (2 * (src + D) - src - rec) * dx / c
    n_steps = int(np.ceil((travel + 10.0 * sigma) / dt))
    n_short = src + D + P
    n_long = n_short + int(np.ceil(n_steps * cfl / 2.0)) + P + 8
    shapes = [(n_short, 1, 1), (n_long, 1, 1)] * n_tab
    nd = 2 * n_tab
    sim = Simulation(1, shapes, dx, dt, nmech, P)
    try:
        sim.set_media([np.zeros(s[0], np.uint8) for s in shapes], np.repeat(np.arange(n_tab), 2),
                      np.full(n_tab, c), np.full(n_tab, rho), np.zeros(n_tab))
        sim.set_relaxation_table(kappa, d, alpha)
        sim.set_sources(np.arange(nd), np.full(nd, src), np.zeros(nd), tone_burst(n_steps, dt, f0, n_cycles)[None, :])
        sim.set_receivers(np.arange(nd), np.full(nd, rec), n_steps)
        sim.step(n_steps)
        tr = sim.read_receivers().astype(np.float64)
    finally:
        sim.close()
    short, long_ = tr[:, 0::2], tr[:, 1::2]
    refl = np.abs(short - long_).max(axis=0)
    inc = np.abs(long_).max(axis=0)
    return 20.0 * np.log10(np.maximum(refl, 1e-300) / inc)


def two_layer_validation(layers, c=1540.0, rho=1000.0, f_pulse=5e6, n_cycles=3, ppw=16, f_top=20e6, cfl=0.2,
                         step_match=True):
    """Two-layer check of Sec. 4 (equal c and rho, different power laws).

    layers: list of pairs ((kappa, d, alpha) of layer 1, (kappa, d, alpha) of
    layer 2), fitted tables.  Per pair, three 1D domains run in one batched
    launch: a two-layer domain with the broadband source, in which the
    two-receiver attenuation is measured inside each layer (receivers at
    0.05 D and 0.8 D from the source, and from the interface, per frequency);
    and a two-layer and a homogeneous layer-1 domain with a Gaussian pulse at
    f_pulse, whose difference at a receiver between source and interface is
    the wave reflected by the interface.  Returns per pair a dict with the
    measured alpha [2][8] and c [2][8] of the layers and R_db =
    20 log10(max|reflected| / max|incident|)."""
    from .sim import Simulation
    dx = c / (ppw * f_top)
    dt = cfl * dx / c
    P, src = 24, 64
    pairs = measurement_cells(dx, c, 0)                      # offsets from a start cell
    x_if = src + int(pairs.max()) + 136                      # first cell of layer 2
    x_refl = x_if - 300                                      # receiver of the reflection domains
    n = x_if + int(pairs.max()) + 200 + P
    n_steps = int(round((x_if + int(pairs.max()) - src) * dx / c / dt)) + 2000
    tabs = []
    for l1, l2 in layers:
        for k, d_, a_ in (l1, l2):
            k, d_, a_ = (np.asarray(v, dtype=np.float64)[None] for v in (k, d_, a_))
            if step_match:
                k, d_, a_ = relax.step_matched(k, d_, a_, dt)
            tabs.append((k[0], d_[0], a_[0]))
    n_pair = len(layers)
    nd = 3 * n_pair
    maps, base = [], []
    two = np.zeros(n, np.uint8)
    two[x_if:] = 1
    for j in range(n_pair):
        maps += [two, two, np.zeros(n, np.uint8)]
        base += [2 * j] * 3
    rec_att = np.unique(np.concatenate([src + pairs.ravel(), x_if + pairs.ravel()]))
    rd, rc = [], []
    for j in range(n_pair):
        rd += [3 * j] * rec_att.size + [3 * j + 1, 3 * j + 2]
        rc += list(rec_att) + [x_refl, x_refl]
    waves = np.stack([broadband_pulse(n_steps, dt), tone_burst(n_steps, dt, f_pulse, n_cycles)])
    sim = Simulation(1, [(n, 1, 1)] * nd, dx, dt, tabs[0][1].shape[1], P)
    try:
        sim.set_media(maps, base, np.full(2 * n_pair, c), np.full(2 * n_pair, rho), np.zeros(2 * n_pair))
        sim.set_relaxation_table(np.array([t[0] for t in tabs]), np.array([t[1] for t in tabs]),
                                 np.array([t[2] for t in tabs]))
        sim.set_sources(np.arange(nd), np.full(nd, src), np.array([0, 1, 1] * n_pair), waves)
        sim.set_receivers(np.array(rd), np.array(rc), n_steps)
        sim.step(n_steps)
        tr = sim.read_receivers().astype(np.float64)
    finally:
        sim.close()
    out = []
    stride = rec_att.size + 2
    col = {int(v): i for i, v in enumerate(rec_att)}
    for j in range(n_pair):
        t = tr[:, j * stride:(j + 1) * stride]
        alpha = np.zeros((2, len(MEASURE_FREQS)))
        cph = np.zeros_like(alpha)
        for layer, start in enumerate((src, x_if)):
            for k, f in enumerate(MEASURE_FREQS):
                a, b = col[start + int(pairs[k, 0])], col[start + int(pairs[k, 1])]
                dist = (pairs[k, 1] - pairs[k, 0]) * dx
                P2 = spectra(t[:, [a, b]], dt, [f])[0]
                al, cc = two_receiver_figures(P2[:1], P2[1:], dist, f, c)
                alpha[layer, k], cph[layer, k] = al[0], cc[0]
        refl = np.abs(t[:, -2] - t[:, -1]).max()
        out.append(dict(alpha=alpha, c=cph, R_db=float(20.0 * np.log10(max(refl, 1e-300) / np.abs(t[:, -1]).max())),
                        interface_cell=x_if, reflection_receiver=x_refl, n_steps=n_steps, dx=dx, dt=dt))
    return out
