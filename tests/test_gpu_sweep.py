"""1D plane-wave sweep (544 domains, alpha0 x y grid) in one batched launch,
with N = 2 relaxation mechanisms (the count the paper validates) and again
with N = 4: simulated attenuation and dispersion against the power law and
the Kramers-Kronig phase velocity, measured as in Sec. 4.1-4.2 (two
receivers at 0.05 D and 0.8 D, D = 10 wavelengths, 8 centre frequencies
1-20 MHz)."""
import numpy as np
import pytest

from workloads import configs
from workloads.adapters import to_simulation
from reporting import report, save

pytestmark = pytest.mark.gpu


def measure(case, traces):
    """Per domain: simulated alpha (Np/m) and phase speed (m/s) at the 8
    measurement frequencies from the receivers at 0.05 D and 0.8 D of each
    frequency (spectra: DFT evaluated at exactly that frequency)."""
    from oracle import analytic
    nd = len(case.shapes)
    rec_cells = list(case.rec_cell[case.rec_domain == 0])
    src = int(case.src_cell[0])
    pairs = configs.sweep_receiver_cells(case.dx, case.c[0], src)
    t = (np.arange(traces.shape[0]) + 1.0) * case.dt
    alpha = np.zeros((nd, len(configs.SWEEP_FREQS)))
    cph = np.zeros_like(alpha)
    c0 = case.c[0]
    for k, fk in enumerate(configs.SWEEP_FREQS):
        ia, ib = rec_cells.index(pairs[k, 0]), rec_cells.index(pairs[k, 1])
        dist = (pairs[k, 1] - pairs[k, 0]) * case.dx
        kern = np.cos(2 * np.pi * fk * t) - 1j * np.sin(2 * np.pi * fk * t)
        for dom in range(nd):
            cols = np.nonzero(case.rec_domain == dom)[0]
            P1 = kern @ traces[:, cols[ia]].astype(np.float64)
            P2 = kern @ traces[:, cols[ib]].astype(np.float64)
            alpha[dom, k] = analytic.two_receiver_attenuation(P1, P2, dist)
            ph = -np.angle(P2 / P1)
            kc = 2 * np.pi * fk / c0
            ph = ph + 2 * np.pi * np.round((kc * dist - ph) / (2 * np.pi))
            cph[dom, k] = 2 * np.pi * fk * dist / ph
    return alpha, cph


@pytest.mark.parametrize("nmech", [2, 4])
def test_sweep_attenuation_and_dispersion(nmech):
    from oracle import analytic
    from paper_2606_11103_amd import relax
    case = configs.sweep_1d(nmech=nmech)
    try:
        kappa, d, al, fits = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), case.nmech,
                                              allow_fit=False, dt=case.dt)
    except KeyError:
        if nmech == 2:
            raise
        pytest.skip("N = %d sweep tables not in the cache (python -m paper_2606_11103_amd.relax_cache --sweep4)"
                    % nmech)
    configs.with_table(case, kappa, d, al)
    print("sweep", len(case.shapes), "domains x", case.shapes[0][0], "cells,", case.n_steps, "steps", flush=True)
    sim = to_simulation(case)
    sim.step(case.n_steps)
    traces = sim.read_receivers()
    assert np.all(np.isfinite(traces))
    alpha, cph = measure(case, traces)
    nrmse, disp = [], []
    valid = np.array([not ft["failed"] for ft in fits])
    for dom in range(len(case.shapes)):
        target = analytic.power_law_alpha(configs.SWEEP_FREQS, case.alpha0[dom], case.y[dom])
        nrmse.append(analytic.nrmse(alpha[dom], target))
        c_kk = 1.0 / analytic.kk_inv_phase_velocity(configs.SWEEP_FREQS, case.c[dom], 1e6, case.alpha0[dom],
                                                    case.y[dom])
        disp.append(np.sqrt(np.mean((cph[dom] - c_kk) ** 2)))
    nrmse, disp = np.array(nrmse), np.array(disp)
    ok = valid & (nrmse <= 0.10) & (disp <= 5.0)
    core = ok & (case.y >= 0.7 - 1e-9) & (case.y <= 1.4 + 1e-9)
    save("sweep_nrmse.npy" if nmech == 2 else "sweep_nrmse_N%d.npy" % nmech,
         np.stack([case.alpha0, case.y, nrmse, disp, valid]))
    report("sweep 544x8192 N=%d: valid %d/%d, NRMSE mean %.4f sd %.4f (core y 0.7-1.4: %.4f), "
            "dispersion RMSE mean %.3f sd %.3f m/s" % (nmech, ok.sum(), len(ok), nrmse[ok].mean(), nrmse[ok].std(),
                                                    nrmse[core].mean(), disp[ok].mean(), disp[ok].std()))
    assert ok.sum() >= 0.7 * len(ok)
    assert nrmse[ok].mean() < 0.03
    assert nrmse[core].mean() < 0.03
    assert disp[ok].mean() < 5.0
