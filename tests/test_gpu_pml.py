"""CPML reflection across tissue tables (the Sec. 4 protocol: 1D plane wave,
1 MHz, 16 points per wavelength, CFL 0.2, D = 5 wavelengths, receiver at
0.8 D, layer 3 wavelengths thick), every table in one batched launch.  The
library's figures are checked against the same protocol run on the FP64
oracle for two tables, and every table must stay below the -50 dB target."""
import numpy as np
import pytest

from oracle.solver import OracleSim
from paper_2606_11103_amd import calibrate, relax
from reporting import report

pytestmark = pytest.mark.gpu


def _oracle_reflection(kappa, d, al, c=1540.0, f0=1e6, ppw=16, cfl=0.2, pmlw=3.0, Dw=5.0, nc=3):
    """The protocol written out independently, run on the FP64 oracle."""
    lam = c / f0
    dx = lam / ppw
    dt = cfl * dx / c
    P, D = int(round(pmlw * ppw)), int(round(Dw * ppw))
    src = P + 4
    rec = src + int(round(0.8 * D))
    sigma = nc / (2 * f0)
    n = int(np.ceil(((2 * (src + D) - src - rec) * dx / c + 10 * sigma) / dt))
    t = (np.arange(n) + 1.0) * dt - 4 * sigma
    w = (np.sin(2 * np.pi * f0 * t) * np.exp(-(t / sigma) ** 2)).astype(np.float32).astype(np.float64)
    n_short = src + D + P
    out = []
    for L in (n_short, n_short + n + P):
        sim = OracleSim(1, (L, 1, 1), dx, dt, len(d[0]), np.zeros(L, np.uint8), [c], [1000.0], [0.0], [kappa],
                        np.array([d]), np.array([al]), pml_cells=P, pml_c_ref=c)
        r, _ = sim.run(n, [src], w[None, :], [rec])
        out.append(r[:, 0])
    return 20 * np.log10(np.abs(out[0] - out[1]).max() / np.abs(out[1]).max())


def test_pml_reflection_over_tissue_tables():
    """Every cached table (grouped by mechanism count and speed), plus a
    lossless one."""
    cache = relax.load_cache()
    groups = {}
    for key, f in sorted(cache.items()):
        groups.setdefault((f["nmech"], f["c"]), []).append(f)
    assert groups, "no cached tables"
    allR, checked = [], 0
    for (N, c), fits in sorted(groups.items()):
        k = np.array([f["kappa"] for f in fits] + [[1.0, 1.0]])
        d = np.array([f["d"] for f in fits] + [np.zeros((2, N))])
        al = np.array([f["alpha"] for f in fits] + [np.full((2, N), 1e8)])
        R = calibrate.pml_reflection(k, d, al, c=c)
        if checked < 3:
            Ro = _oracle_reflection(k[0], d[0], al[0], c=c)
            assert abs(R[0] - Ro) < 1.0, (R[0], Ro)
            checked += 1
        allR.append(R[:-1])
        assert R[-1] < -50.0
    allR = np.concatenate(allR)
    report("CPML reflection (3 wavelengths, 1 MHz) over %d tissue tables: median %.1f dB, max %.1f dB, "
            "below -50 dB: %d/%d" % (allR.size, np.median(allR), allR.max(), int((allR < -50).sum()), allR.size))
    assert np.all(allR < -50.0)
