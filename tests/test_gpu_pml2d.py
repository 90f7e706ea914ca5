"""The Sec. 4.3 reflection protocol in 2D (plane wave, 1 MHz, 16 points per
wavelength, CFL 0.2, D = 5 and W = 20 wavelengths, 3-wavelength layers)
for the four bottom-layer designs of paper_2606_11103_amd.pml, over every
cached tissue table in batched 2D launches, with step-matched and with
paper-literal (unmatched) tables; one table per design checked against the
same protocol run on the FP64 oracle."""
import os

import numpy as np
import pytest

from oracle.solver import OracleSim
from paper_2606_11103_amd import pml, relax
from reporting import report

pytestmark = pytest.mark.gpu


# every cached table with FW25_FULL_SWEEPS=1 (1644 tables, about 25 s per
# design and table variant); by default every sixth table of the two large
# groups and all others (about 300), which keeps the figures within 1 dB
FULL = os.environ.get("FW25_FULL_SWEEPS") == "1"


def _groups():
    cache = relax.load_cache()
    groups = {}
    for key, f in sorted(cache.items()):
        groups.setdefault((f["nmech"], f["c"]), []).append(f)
    assert groups, "no cached tables"
    if not FULL:
        groups = {k: (v if len(v) < 50 else v[::6]) for k, v in groups.items()}
    return groups


def _reference(N):
    """The homogeneous layers' fixed tissue: the cached fit of (alpha0, y) =
    (0.5, 1.0) at c = 1540 with N mechanisms."""
    cache = relax.load_cache()
    key = relax._key(1540.0, 0.5, 1.0, N, 50000)
    if key not in cache:
        pytest.skip("no cached fit of the reference tissue (0.5, 1.0), N=%d" % N)
    f = relax.effective(cache[key])
    return np.array(f["kappa"]), np.array(f["d"]), np.array(f["alpha"])


def _oracle_reflection(k, d, al, design, ref, g, c=1540.0):
    """The protocol of pml.reflection_2d for one table run on the FP64
    oracle, with the geometry, waveform and class tables of the library run g."""
    ks, ds, als = g["tables"]
    nx, (ny_s, ny_l) = g["nx"], g["ny"]
    out = []
    for ny, first in ((ny_s, True), (ny_l, False)):
        lab = np.zeros((ny, nx), np.uint8)
        if first:
            _, _, _, rows = pml.bottom_layer_tables(k, d, al, design, g["LT"], g["P"], ref)
            lab[ny - g["LT"] - g["P"]:, :] = rows.astype(np.uint8)[:, None]
        n_cls = int(lab.max()) + 1 if first else 1
        sim = OracleSim(2, (nx, ny, 1), g["dx"], g["dt"], d.shape[1], lab, [c] * n_cls, [1000.0] * n_cls,
                        [0.0] * n_cls, ks[:n_cls], ds[:n_cls], als[:n_cls], pml_cells=g["P"], pml_c_ref=c)
        src = g["src"] * nx + np.arange(nx)
        r, _ = sim.run(g["n_steps"], src, np.repeat(g["wave"].astype(np.float64)[None, :], nx, 0),
                       [g["rec"] * nx + nx // 2])
        out.append(r[:, 0])
    return 20 * np.log10(np.abs(out[0] - out[1]).max() / np.abs(out[1]).max())


@pytest.mark.parametrize("design", pml.DESIGNS)
def test_design_matches_oracle_for_one_table(design):
    ref = _reference(2)
    cache = relax.load_cache()
    f = relax.effective(cache[relax._key(1540.0, 0.5, 1.1, 2, 50000)])   # the 2D homogeneous workload's tissue
    k, d, al = np.array(f["kappa"]), np.array(f["d"]), np.array(f["alpha"])
    R, g = pml.reflection_2d(k[None], d[None], al[None], design=design, ref=ref, step_match=False,
                             return_traces=True)
    R = R[0]
    Ro = _oracle_reflection(k, d, al, design, ref, g)
    report("2D reflection, design %s, tissue (0.5, 1.1) N=2: library %.2f dB, FP64 oracle %.2f dB" % (design, R, Ro))
    assert abs(R - Ro) < 0.5


@pytest.mark.parametrize("step_match", [True, False], ids=["step_matched", "paper_literal"])
@pytest.mark.parametrize("design", pml.DESIGNS)
def test_reflection_over_tissue_tables(design, step_match):
    allR = []
    for (N, c), fits in sorted(_groups().items()):
        k = np.array([f["kappa"] for f in fits])
        d = np.array([f["d"] for f in fits])
        al = np.array([f["alpha"] for f in fits])
        ref = _reference(N) if design.startswith("homog") else None
        print("design", design, "N", N, "c", c, "tables", len(fits), flush=True)
        allR.append(pml.reflection_2d(k, d, al, design=design, ref=ref, c=c, step_match=step_match))
    R = np.concatenate(allR)
    st = pml.stats(R)
    report("2D reflection, design %s, %s tables: %d tables, median %.1f dB, worst %.1f dB, below -50 dB %.1f %%, "
           "diverged %d" % (design, "step-matched" if step_match else "paper-literal", st["n"], st["median"],
                            st["worst"], 100 * st["frac_below"], st["diverged"]))
    # measured (1644 tables): composed median -80.9 dB, worst -79.2; two-stage
    # median -104.7, worst -77.7; the fixed-tissue layers (with or without the
    # transition region) median -51.2 dB, 55 % below -50 dB, worst -29.6
    assert st["diverged"] == 0
    if design == "composed":
        assert st["worst"] < -70.0 and st["median"] < -75.0
    elif design == "two_stage":
        assert st["worst"] < -70.0 and st["median"] < -95.0
    else:
        # a layer holding one fixed tissue reflects at the tissue mismatch far
        # above the adaptive layers (Sec. 5.5 finds the same ordering)
        assert st["median"] > -60.0 and st["frac_below"] < 0.9
