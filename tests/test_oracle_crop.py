"""The oracle on a crop equals the oracle on the whole domain while the
field has not reached the crop's edges (CPU, no GPU): pins the crop set-up
used by the full-size parity test (full-domain noise index, CPML profiles
restricted to the crop)."""
import numpy as np

from workloads import configs
from workloads.adapters import to_oracle, to_oracle_crop


def test_crop_equals_full_domain_before_the_field_reaches_its_edges():
    case = configs.heterogeneous_3d(shape=(96, 80, 72), steps=40, n_elem=8)
    configs.with_table(case, *configs.random_relaxation_table(3, case.n_classes, case.nmech))
    K = 4
    full = to_oracle(case)
    w = case.waves.astype(np.float64)[case.src_wave]
    full.run(K, case.src_cell, w, [])
    nx, ny, nz = case.shapes[0]
    sx = case.src_cell % nx
    sy = (case.src_cell // nx) % ny
    sz = case.src_cell // (nx * ny)
    m = 8 * K + 8
    lo = [max(0, sx.min() - m), max(0, sy.min() - m), 0]
    hi = [min(nx, sx.max() + 1 + m), min(ny, sy.max() + 1 + m), min(nz, sz.max() + 1 + m)]
    crop = to_oracle_crop(case, lo, hi)
    lx, ly = hi[0] - lo[0], hi[1] - lo[1]
    local = ((sz - lo[2]) * ly + (sy - lo[1])) * lx + (sx - lo[0])
    crop.run(K, local, w, [])
    pf = full.p.reshape(nz, ny, nx)
    pc = crop.p.reshape(hi[2] - lo[2], ly, lx)
    assert np.abs(pf).max() > 0
    np.testing.assert_array_equal(pf[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]], pc)
    inside = np.zeros_like(pf, dtype=bool)
    inside[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
    assert np.all(pf[~inside] == 0)
