"""Weight selection by simulated attenuation (Sec. 3.2) on the GPU: every
objective weight's parameter set of every sweep class runs as one domain of
a single batched 1D launch, and each class keeps the weight whose simulated
attenuation NRMSE (Sec. 4.1) is lowest."""
import numpy as np
import pytest

from oracle import analytic
from paper_2606_11103_amd import calibrate, relax
from workloads import configs
from reporting import report, save

pytestmark = pytest.mark.gpu


def _independent_measure(run, traces):
    """Two-receiver figures written out with the oracle's Sec. 4.1 formula and
    a plain DFT loop per frequency and domain."""
    t = (np.arange(traces.shape[0]) + 1.0) * run.dt
    cells = list(run.cells)
    alpha = np.zeros((run.n_dom, 8))
    cph = np.zeros((run.n_dom, 8))
    for k, f in enumerate(configs.SWEEP_FREQS):
        ia, ib = cells.index(run.pairs[k, 0]), cells.index(run.pairs[k, 1])
        dist = (run.pairs[k, 1] - run.pairs[k, 0]) * run.dx
        kern = np.cos(2 * np.pi * f * t) - 1j * np.sin(2 * np.pi * f * t)
        for j in range(run.n_dom):
            P1 = kern @ traces[:, j, ia].astype(np.float64)
            P2 = kern @ traces[:, j, ib].astype(np.float64)
            alpha[j, k] = analytic.two_receiver_attenuation(P1, P2, dist)
            ph = -np.angle(P2 / P1)
            ph = ph + 2 * np.pi * np.round((2 * np.pi * f / run.c * dist - ph) / (2 * np.pi))
            cph[j, k] = 2 * np.pi * f * dist / ph
    return alpha, cph


def _discrete_figures(run, kappa, d, al):
    """Attenuation and phase speed of the discrete scheme itself (exact 1D
    complex wavenumber of the leapfrog staggered scheme with the recursions'
    frequency response), from the oracle's closed forms."""
    from oracle import fdcoef
    w = 2 * np.pi * configs.SWEEP_FREQS
    S = []
    for i in range(2):
        a, b = analytic.recursion_coefficients(kappa[i], np.asarray(d[i]), np.asarray(al[i]), run.dt)
        S.append(analytic.discrete_stretch(w, kappa[i], a, b, run.dt))
    k = analytic.discrete_wavenumber(configs.SWEEP_FREQS, run.c, run.dx, run.dt, fdcoef.staggered_coefficients(4),
                                     S[0], S[1])
    return -k.imag, w / k.real


def test_simulated_attenuation_of_soft_tissue_class():
    """The cached N = 2 fit of (c 1540, alpha0 0.5, y 1.1), step-matched to
    the run's time step, and a lossless table in one batched 1D run with CPML
    at both ends: the library's two-receiver measurement equals an
    independent one; both domains follow the scheme's exact discrete
    wavenumber (so the CPML leaves the measurement untouched); the lossy
    class follows the power law within the 3 % bar."""
    key = [k for k in relax.load_cache() if k.startswith("c=1540.000000|a0=0.5|y=1.100000|N=2")]
    assert key, "cached fit of the soft-tissue class is missing"
    ft = relax.load_cache()[key[0]]
    kappa = np.array([ft["kappa"], [1.0, 1.0]])
    d = np.array([ft["d"], np.zeros((2, 2))])
    al = np.array([ft["alpha"], np.full((2, 2), 1e8)])
    run = calibrate.SweepRun(kappa, d, al)
    print("calibration run", run.n_dom, "domains", run.n_steps, "steps", flush=True)
    tr = run.run()
    a, c = run.measure(tr)
    ai, ci = _independent_measure(run, tr)
    np.testing.assert_allclose(a, ai, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(c, ci, rtol=1e-12)
    nr, disp = calibrate.errors(a[0], c[0], 1540.0, 0.5, 1.1)
    ad, cd = _discrete_figures(run, run.kappa[0], run.d[0], run.alpha[0])
    a0d, c0d = _discrete_figures(run, run.kappa[1], run.d[1], run.alpha[1])
    report("calibration soft tissue N=2: simulated NRMSE %.4f dispersion %.3f m/s; vs discrete scheme: "
            "alpha max rel %.2e, c max %.3f m/s; lossless max |alpha| %.3g Np/m, max |c - c_discrete| %.3g m/s"
            % (nr, disp, np.max(np.abs(a[0] / ad - 1)), np.abs(c[0] - cd).max(), np.abs(a[1]).max(),
               np.abs(c[1] - c0d).max()))
    assert np.max(np.abs(a[0] / ad - 1)) < 5e-3
    assert np.abs(c[0] - cd).max() < 0.1
    assert np.abs(a[1]).max() < 0.1
    assert np.abs(c[1] - c0d).max() < 0.1
    assert nr < 0.03 and disp < 2.0


def _selection_stats(fits, nr, dp):
    """Per class: the candidate chosen on the simulated figures and the one
    chosen on the closed-form figures, with their simulated NRMSE."""
    j_sim = np.array([relax.choose(f["cands"], nr[i], dp[i]) for i, f in enumerate(fits)])
    j_mod = np.array([relax.choose(f["cands"]) for f in fits])
    rows = np.arange(len(fits))
    ok = np.array([relax.passes(nr[i, j], dp[i, j]) for i, j in enumerate(j_sim)])
    return j_sim, j_mod, nr[rows, j_sim], nr[rows, j_mod], dp[rows, j_sim], ok


@pytest.mark.parametrize("nmech", [2, 4])
def test_weight_selection_over_the_sweep(nmech):
    case = configs.sweep_1d(n_cells=64, steps=10, pml=8)
    cache = relax.load_cache()
    keys = [relax._key(c, a0, y, nmech, 50000) for c, a0, y in zip(case.c, case.alpha0, case.y)]
    if any(k not in cache or "cands" not in cache[k] for k in keys):
        pytest.skip("sweep fits with per-weight candidates are not cached")
    fits = [relax.effective(cache[k]) for k in keys]
    chosen, nr, dp = calibrate.select_weights(fits)
    j_sim, j_mod, nr_sim, nr_mod, dp_sim, ok = _selection_stats(fits, nr, dp)
    assert np.array_equal(j_sim, [[cd["w"] for cd in f["cands"]].index(c["w"]) for f, c in zip(fits, chosen)])
    ok_mod = np.array([relax.passes(nr[i, j], dp[i, j]) for i, j in enumerate(j_mod)])
    report("weight selection N=%d, %d classes x %d weights: within both bars %d (closed-form choice: %d), "
            "simulated NRMSE mean %.4f sd %.4f (closed-form choice %.4f), dispersion mean %.3f m/s"
            % (nmech, len(fits), nr.shape[1], ok.sum(), ok_mod.sum(), nr_sim[ok].mean(), nr_sim[ok].std(),
               nr_mod[ok_mod].mean(), dp_sim[ok].mean()))
    save("weight_selection.npy" if nmech == 2 else "weight_selection_N%d.npy" % nmech,
         np.stack([case.alpha0, case.y, nr_sim, nr_mod, ok]))
    # floors a few cells under the measured figures (N = 2: 504 of 544 within
    # both bars, mean 1.19 %; N = 4: 507, 1.21 %), so that a regression of
    # the fits, the batched 1D launch or the measurement shows; selection by
    # simulation never passes fewer cells than the closed-form choice
    floor = {2: 500, 4: 503}[nmech]
    assert ok.sum() >= floor
    assert ok.sum() >= ok_mod.sum()
    assert nr_sim[ok].mean() < 0.014


def test_weight_selection_over_the_library():
    """The 1071-cell (alpha0, y) relaxation library, every weight's candidate
    simulated in one batched launch (5355 domains), each cell keeping the
    weight chosen on its simulated figures.  Reported beside the paper's
    heat-map statistics (Sec. 4, 1328 cells: 2.61 % +- 1.83 %)."""
    lib = configs.library_classes()
    cache = relax.load_cache()
    keys = [relax._key(c, a0, y, 2, 50000) for c, a0, y in zip(lib["c"], lib["alpha0"], lib["y"])]
    if any(k not in cache or "cands" not in cache[k] for k in keys):
        pytest.skip("library fits with per-weight candidates are not cached")
    fits = [relax.effective(cache[k]) for k in keys]
    chosen, nr, dp = calibrate.select_weights(fits)
    j_sim, j_mod, nr_sim, nr_mod, dp_sim, ok = _selection_stats(fits, nr, dp)
    core = ok & (lib["y"] >= 0.7 - 1e-9) & (lib["y"] <= 1.4 + 1e-9)
    report("relaxation library %d cells x %d weights: within both bars %d, simulated NRMSE mean %.4f sd %.4f "
            "(core y 0.7-1.4: %.4f), dispersion mean %.3f sd %.3f m/s (paper: 1328 cells, 2.61 %% +- 1.83 %%, "
            "1.14 +- 0.76 m/s)" % (len(fits), nr.shape[1], ok.sum(), nr_sim[ok].mean(), nr_sim[ok].std(),
                                   nr_sim[core].mean(), dp_sim[ok].mean(), dp_sim[ok].std()))
    save("library_selection.npy", np.stack([lib["alpha0"], lib["y"], nr_sim, dp_sim, ok]))
    assert ok.sum() >= 0.7 * len(fits)
    assert nr_sim[ok].mean() < 0.03


def test_two_layer_tissue_pairs():
    """Sec. 4 two-layer check (c and rho equal across the interface): muscle
    (alpha0 0.15, y 1.0), fat (0.40, 1.1) and liver (0.50, 1.1) in the pairs
    the paper uses.  Per-layer attenuation NRMSE against each layer's power
    law, and the interface reflection of a 5 MHz pulse; the reflection of one
    pair is recomputed on the FP64 oracle."""
    from oracle.solver import OracleSim
    cache = relax.load_cache()
    tissues = {"muscle": (0.15, 1.0), "fat": (0.40, 1.1), "liver": (0.50, 1.1)}
    fits = {}
    for name, (a0, y) in tissues.items():
        f = cache.get(relax._key(1540.0, a0, y, 2, 50000))
        if f is None:
            pytest.skip("tissue fits not cached")
        fits[name] = f
    order = [("muscle", "fat"), ("muscle", "liver"), ("fat", "liver")]
    paper = {("muscle", "fat"): (1.18, 0.847, -63.0), ("muscle", "liver"): (1.18, 1.41, -50.2),
             ("fat", "liver"): (0.978, 2.32, -50.5)}
    tab = lambda f: (f["kappa"], f["d"], f["alpha"])
    res = calibrate.two_layer_validation([(tab(fits[a]), tab(fits[b])) for a, b in order])
    for (a, b), r in zip(order, res):
        nr = [calibrate.errors(r["alpha"][i], r["c"][i], 1540.0, *tissues[t])[0] for i, t in enumerate((a, b))]
        report("two-layer %s -> %s: NRMSE layer 1 %.2f %% layer 2 %.2f %%, interface reflection %.1f dB "
                "(paper: %.2f %%, %.2f %%, %.1f dB)" % (a, b, 100 * nr[0], 100 * nr[1], r["R_db"], *paper[(a, b)]))
        assert max(nr) < 0.03
        assert r["R_db"] < -40.0
    # FP64 oracle: the muscle -> liver reflection with the same tables and geometry
    r = res[1]
    k, d, al = relax.step_matched(np.array([fits["muscle"]["kappa"], fits["liver"]["kappa"]]),
                                  np.array([fits["muscle"]["d"], fits["liver"]["d"]]),
                                  np.array([fits["muscle"]["alpha"], fits["liver"]["alpha"]]), r["dt"])
    n = r["interface_cell"] + 2560 + 200 + 24
    t = (np.arange(r["n_steps"]) + 1.0) * r["dt"] - 4 * (3 / (2 * 5e6))
    w = (np.sin(2 * np.pi * 5e6 * t) * np.exp(-(t / (3 / (2 * 5e6))) ** 2)).astype(np.float32).astype(np.float64)
    out = []
    for two in (True, False):
        cm = np.zeros(n, np.uint8)
        if two:
            cm[r["interface_cell"]:] = 1
        sim = OracleSim(1, (n, 1, 1), r["dx"], r["dt"], 2, cm, [1540.0, 1540.0], [1000.0, 1000.0], [0.0, 0.0],
                        k, d, al, pml_cells=24, pml_c_ref=1540.0)
        tr, _ = sim.run(r["n_steps"], [64], w[None, :], [r["reflection_receiver"]])
        out.append(tr[:, 0])
    R_or = 20 * np.log10(np.abs(out[0] - out[1]).max() / np.abs(out[1]).max())
    report("two-layer muscle -> liver reflection: library %.2f dB, FP64 oracle %.2f dB" % (r["R_db"], R_or))
    assert abs(r["R_db"] - R_or) < 1.0


@pytest.mark.parametrize("which", ["sweep", "library"])
def test_paper_literal_and_step_matched_tables(which):
    """The simulated attenuation and dispersion of every cached fit of the
    544-cell sweep or the 1071-cell library (N = 2, closed-form weight
    choice), run as fitted (paper-literal: the continuous model's mechanisms
    straight into the recursion) and step-matched to the run's time step
    (16 points per wavelength at 20 MHz, CFL 0.2), both in one batched 1D
    launch each, beside the paper's 2.61 % +- 1.83 % and 1.14 +- 0.76 m/s."""
    if which == "sweep":
        case = configs.sweep_1d(n_cells=64, steps=10, pml=8)
        cls = dict(c=case.c, alpha0=case.alpha0, y=case.y)
    else:
        cls = configs.library_classes()
    cache = relax.load_cache()
    keys = [relax._key(c, a0, y, 2, 50000) for c, a0, y in zip(cls["c"], cls["alpha0"], cls["y"])]
    if any(k not in cache for k in keys):
        pytest.skip("%s fits are not cached" % which)
    fits = [relax.effective(cache[k]) for k in keys]
    out = {}
    for matched in (False, True):
        run = calibrate.SweepRun([f["kappa"] for f in fits], [f["d"] for f in fits], [f["alpha"] for f in fits],
                                 step_match=matched)
        a, c = run.measure(run.run())
        nr = np.zeros(len(fits))
        dp = np.zeros(len(fits))
        for i, f in enumerate(fits):
            nr[i], dp[i] = calibrate.errors(a[i], c[i], f["c"], f["alpha0"], f["y"])
        ok = np.array([relax.passes(nr[i], dp[i]) for i in range(len(fits))])
        core = ok & (np.asarray(cls["y"]) >= 0.7 - 1e-9) & (np.asarray(cls["y"]) <= 1.4 + 1e-9)
        out[matched] = (nr, dp, ok)
        report("%s %d cells, %s tables: within both bars %d, NRMSE over those %.2f %% +- %.2f %% (core y 0.7-1.4: "
               "%.2f %%), over all cells %.2f %% +- %.2f %%; dispersion RMSE %.2f +- %.2f m/s (paper: 1328 cells, "
               "2.61 %% +- 1.83 %%, 1.14 +- 0.76 m/s)"
               % (which, len(fits), "step-matched" if matched else "paper-literal", ok.sum(), 100 * nr[ok].mean(),
                  100 * nr[ok].std(), 100 * nr[core].mean(), 100 * nr.mean(), 100 * nr.std(), dp[ok].mean(),
                  dp[ok].std()))
        save("%s_%s.npy" % (which, "matched" if matched else "literal"),
             np.stack([np.asarray(cls["alpha0"]), np.asarray(cls["y"]), nr, dp, ok]))
    # mapping the fitted mechanisms to the time step is what brings the
    # scheme onto the fitted model: more cells within the bars, lower error
    assert out[True][2].sum() > out[False][2].sum()
    assert np.mean(out[True][0]) < np.mean(out[False][0])
