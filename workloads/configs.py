"""Seeded synthetic cases: plain arrays consumed by both the product and the
oracle.  No arithmetic of the method lives here (see the package docstring).

A Case holds the grid, the tissue classes (c, rho, alpha0, y, B/A), the class
maps, sources and receivers.  The relaxation table (kappa, d, alpha per class)
is filled in by the caller: from the calibration (bench) or drawn at random
(parity tests, where any admissible table will do).
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import (draw_tissue_classes, gaussian_derivative, layered_labels, linear_index,
               smoothed_label_field, tone_burst)


@dataclasses.dataclass
class Case:
    name: str
    ndim: int
    shapes: List[tuple]                 # (nx, ny, nz) per domain
    dx: float
    dt: float
    nmech: int
    pml_cells: int
    class_maps: List[np.ndarray]        # uint8 (nz, ny, nx) per domain, local indices
    class_base: List[int]
    c: np.ndarray
    rho: np.ndarray
    alpha0: np.ndarray
    y: np.ndarray
    b_over_a: np.ndarray
    nonlinear: bool
    src_domain: np.ndarray
    src_cell: np.ndarray
    src_wave: np.ndarray
    waves: np.ndarray                   # float32 [n_wave][n_t]
    rec_domain: np.ndarray
    rec_cell: np.ndarray
    n_steps: int
    noise_amp: float = 0.0
    noise_seed: int = 0
    pml_params: Optional[tuple] = None  # (R0, f_alpha, c_ref)
    kappa: Optional[np.ndarray] = None  # [C][2]
    d: Optional[np.ndarray] = None      # [C][2][N]
    alpha: Optional[np.ndarray] = None  # [C][2][N]
    strength: Optional[List[np.ndarray]] = None   # per-voxel strength scale in [0, 1] per domain (float32)
    fd_c_ref: float = 0.0               # > 0: staggered coefficients of the time-space set for this speed
    fd_widened: bool = False            # with fd_c_ref, 2D: the widened (off-axis) stencil

    @property
    def n_classes(self):
        return len(self.c)

    def cells(self):
        return sum(int(np.prod(s)) for s in self.shapes)


def random_relaxation_table(seed, n_classes, nmech):
    """Admissible relaxation parameters like those the calibration returns:
    kappa in [0.98, 1], alpha log-uniform in [10^6.5, 10^10] and a relaxation
    strength d / (d + kappa alpha) log-uniform in [1e-4, 3e-2] (the range
    fitted tissue classes span), all inside the bounds of Table 2."""
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.98, 1.0, size=(n_classes, 2))
    alpha = 10.0 ** rng.uniform(6.5, 10.0, size=(n_classes, 2, nmech))
    strength = 10.0 ** rng.uniform(-4.0, math.log10(3e-2), size=(n_classes, 2, nmech))
    d = strength * kappa[:, :, None] * alpha / (1.0 - strength)
    return kappa, d, alpha


def with_strength(case, seed, lo=0.2, hi=1.0):
    """Attach a smooth seeded per-voxel strength map to every domain of the
    case (see workloads.smooth_unit_field)."""
    from . import smooth_unit_field
    case.strength = [smooth_unit_field(m.shape, seed + 31 * k, lo, hi) for k, m in enumerate(case.class_maps)]
    return case


def with_table(case, kappa, d, alpha):
    case.kappa = np.asarray(kappa, dtype=np.float64).reshape(case.n_classes, 2)
    case.d = np.asarray(d, dtype=np.float64).reshape(case.n_classes, 2, case.nmech)
    case.alpha = np.asarray(alpha, dtype=np.float64).reshape(case.n_classes, 2, case.nmech)
    return case


# ------------------------------------------------------------ named cases --
def homogeneous_2d(n=256, steps=600):
    """2D homogeneous: 256 x 256 cells, dx = 0.05 mm, c = 1540, rho = 1000,
    alpha0 = 0.5, y = 1.1, N = 2, linear, 20-cell CPML, CFL 0.4, 600 steps;
    point source (3 MHz, 3-cycle Gaussian-windowed) at the centre, receivers
    1 mm and 4 mm from it (3 mm apart)."""
    dx, c = 5e-5, 1540.0
    dt = 0.4 * dx / c
    shp = (n, n, 1)
    ctr = n // 2
    return Case(
        name="2d_homogeneous_%d" % n, ndim=2, shapes=[shp], dx=dx, dt=dt, nmech=2, pml_cells=20,
        class_maps=[np.zeros((1, n, n), np.uint8)], class_base=[0],
        c=np.array([c]), rho=np.array([1000.0]), alpha0=np.array([0.5]), y=np.array([1.1]),
        b_over_a=np.array([0.0]), nonlinear=False,
        src_domain=np.zeros(1, np.int32), src_cell=np.array([linear_index(shp, ctr, ctr)]),
        src_wave=np.zeros(1, np.int32), waves=tone_burst(steps, dt, 3e6, 3)[None, :],
        rec_domain=np.zeros(2, np.int32),
        rec_cell=np.array([linear_index(shp, ctr + 20, ctr), linear_index(shp, ctr + 80, ctr)]),
        n_steps=steps)


def two_layer_2d(n=2048, steps=4000, n_rec=128):
    """2D two-layer: 2048 x 2048 cells, dx = 0.03 mm; interface at the middle
    row; top c = 1580, rho = 1090, alpha0 = 0.9, y = 1.1, B/A = 6; bottom
    c = 1450, rho = 950, alpha0 = 0.4, y = 1.4, B/A = 9; N = 4; 24-cell CPML;
    CFL 0.4 on 1580 m/s; plane-wave line source (5 MHz, 4 cycles, 0.8 MPa)
    along row 28; receivers on the centre column every 15 rows from row 64."""
    dx = 3e-5
    dt = 0.4 * dx / 1580.0
    shp = (n, n, 1)
    lab = layered_labels((1, n, n), [n // 2], axis=1)
    P = 24
    xs = np.arange(P, n - P)
    rows = 64 + 15 * np.arange(n_rec)
    rows = rows[rows < n - P]
    return Case(
        name="2d_two_layer_%d" % n, ndim=2, shapes=[shp], dx=dx, dt=dt, nmech=4, pml_cells=P,
        class_maps=[lab], class_base=[0],
        c=np.array([1580.0, 1450.0]), rho=np.array([1090.0, 950.0]), alpha0=np.array([0.9, 0.4]),
        y=np.array([1.1, 1.4]), b_over_a=np.array([6.0, 9.0]), nonlinear=True,
        src_domain=np.zeros(xs.size, np.int32), src_cell=linear_index(shp, xs, 28),
        src_wave=np.zeros(xs.size, np.int32), waves=tone_burst(steps, dt, 5e6, 4, amplitude=0.8e6)[None, :],
        rec_domain=np.zeros(rows.size, np.int32), rec_cell=linear_index(shp, n // 2, rows),
        n_steps=steps)


def heterogeneous_3d(shape=(960, 960, 720), steps=2000, seed=3, noise_seed=33, n_elem=64, nmech=4):
    """3D heterogeneous: 960 x 960 x 720 cells (z slowest), dx = 0.1 mm,
    24-cell CPML, 8 tissue classes (seed 3) from a smoothed random label field,
    +-1 % per-voxel speed perturbation (SplitMix64 seed 33), N = 4, CFL 0.4 on
    1650 * 1.01 m/s, 2000 steps.  Source: 64-element linear array along x at
    z = 28 (pitch 3 cells, elements 2 x 100 cells) focused at 40 mm depth
    (delays for 1540 m/s), 2.5 MHz, 3 cycles, 0.5 MPa.  Receivers: the 64
    element centres and 64 points on the axis at z = 60 + 10 k (those inside
    the grid)."""
    nx, ny, nz = shape
    dx = 1e-4
    dt = 0.4 * dx / (1650.0 * 1.01)
    P = 24
    cls = draw_tissue_classes(8, seed)
    lab = smoothed_label_field((nz, ny, nx), 8, seed, coarse=4, sigma=5.0)
    zs = min(28, nz // 4)
    cx, cy = nx // 2, ny // 2
    pitch = 3
    elem_y = min(100, max(2, ny - 2 * P - 2))
    n_elem = max(1, min(n_elem, (nx - 2 * P - 2) // pitch))
    x_e = cx - (n_elem * pitch) // 2 + pitch * np.arange(n_elem)
    zf = zs + 400
    dist = np.hypot((x_e + 0.5 - cx) * dx, (zf - zs) * dx)
    delay = (dist.max() - dist) / 1540.0
    waves = np.stack([tone_burst(steps, dt, 2.5e6, 3, amplitude=0.5e6, delay=t) for t in delay])
    sx, sy, sw = [], [], []
    for e in range(n_elem):
        for ddx in range(2):
            for yy in range(cy - elem_y // 2, cy - elem_y // 2 + elem_y):
                sx.append(x_e[e] + ddx)
                sy.append(yy)
                sw.append(e)
    src_cell = linear_index(shape, np.array(sx), np.array(sy), zs)
    rz = 60 + 10 * np.arange(64)
    rz = rz[rz < nz - P]
    rec_cell = np.concatenate([linear_index(shape, x_e, cy, zs), linear_index(shape, cx, cy, rz)])
    return Case(
        name="3d_heterogeneous_%dx%dx%d" % tuple(shape) + ("" if nmech == 4 else "_N%d" % nmech), ndim=3,
        shapes=[tuple(shape)], dx=dx, dt=dt, nmech=nmech,
        pml_cells=P, class_maps=[lab], class_base=[0],
        c=cls["c"], rho=cls["rho"], alpha0=cls["alpha0"], y=cls["y"], b_over_a=cls["b_over_a"], nonlinear=True,
        src_domain=np.zeros(len(sx), np.int32), src_cell=src_cell, src_wave=np.array(sw, np.int32), waves=waves,
        rec_domain=np.zeros(rec_cell.size, np.int32), rec_cell=rec_cell, n_steps=steps,
        noise_amp=0.01, noise_seed=noise_seed)


def random_small(ndim, shapes, nmech, n_classes, seed, steps, pml=6, nonlinear=True, noise=0.01,
                 amplitude=2e5, n_rec=12):
    """Small heterogeneous case for parity tests: random label fields, random
    tissue classes, one point source per domain and scattered receivers."""
    rng = np.random.default_rng(seed)
    cls = draw_tissue_classes(n_classes * len(shapes), seed)
    dx = 1e-4
    cmax = cls["c"].max() * (1 + noise)
    dt = (0.4 if ndim < 3 else 0.35) * dx / cmax
    maps, base = [], []
    sd, sc, rd, rc = [], [], [], []
    for d, shp in enumerate(shapes):
        nx, ny, nz = shp
        lab = rng.integers(0, n_classes, size=(nz, ny, nx)).astype(np.uint8)
        if ndim >= 2:
            lab = smoothed_label_field((nz, ny, nx), n_classes, seed + 17 * d, coarse=2, sigma=1.5)
        maps.append(lab)
        base.append(d * n_classes)
        lo = [pml + 1 if s > 1 else 0 for s in shp]
        hi = [s - pml - 1 if s > 1 else 1 for s in shp]
        p = [int(rng.integers(lo[a], hi[a])) for a in range(3)]
        sd.append(d)
        sc.append(int(linear_index(shp, p[0], p[1], p[2])))
        for _ in range(n_rec):
            q = [int(rng.integers(0, shp[a])) for a in range(3)]
            rd.append(d)
            rc.append(int(linear_index(shp, q[0], q[1], q[2])))
    waves = tone_burst(steps, dt, 2e6, 2, amplitude=amplitude)[None, :]
    return Case(
        name="random_%dd_%d" % (ndim, seed), ndim=ndim, shapes=[tuple(s) for s in shapes], dx=dx, dt=dt,
        nmech=nmech, pml_cells=pml, class_maps=maps, class_base=base,
        c=cls["c"], rho=cls["rho"], alpha0=cls["alpha0"], y=cls["y"], b_over_a=cls["b_over_a"],
        nonlinear=nonlinear, src_domain=np.array(sd, np.int32), src_cell=np.array(sc, np.int64),
        src_wave=np.zeros(len(sd), np.int32), waves=waves, rec_domain=np.array(rd, np.int32),
        rec_cell=np.array(rc, np.int64), n_steps=steps, noise_amp=noise, noise_seed=seed * 7 + 1)


SWEEP_ALPHA0 = 0.0022 * (1.0 / 0.0022) ** (np.arange(32) / 31.0)
SWEEP_Y = 0.4 + 0.1 * np.arange(17)
SWEEP_FREQS = 1e6 + 2.714e6 * np.arange(8)
# relaxation library grid: 63 log-spaced alpha0 (every other one is a sweep
# value) x the 17 sweep exponents = 1071 (alpha0, y) cells
LIBRARY_ALPHA0 = 0.0022 * (1.0 / 0.0022) ** (np.arange(63) / 62.0)
LIBRARY_Y = SWEEP_Y


def library_classes(c=1540.0):
    """dict(c, alpha0, y) of every cell of the relaxation library grid."""
    A0, Y = np.meshgrid(LIBRARY_ALPHA0, LIBRARY_Y, indexing="ij")
    return dict(c=np.full(A0.size, c), alpha0=A0.ravel(), y=Y.ravel())


def sweep_receiver_cells(dx, c=1540.0, src_cell=64, freqs=None):
    """Receiver cells of the two-receiver measurement: for each measurement
    frequency f, the cells nearest 0.05 D and 0.8 D from the source, with
    D = 10 wavelengths at f (Sec. 4.1).  Returns [n_freq][2]."""
    freqs = SWEEP_FREQS if freqs is None else np.asarray(freqs, dtype=np.float64)
    out = []
    for f in freqs:
        D = 10.0 * c / f
        out.append([src_cell + int(round(0.05 * D / dx)), src_cell + int(round(0.8 * D / dx))])
    return np.array(out, dtype=np.int64)


def sweep_1d(n_cells=8192, nmech=2, steps=None, alpha0=None, y=None, c=1540.0, rho=1000.0, pml=24,
             src_cell=64):
    """1D plane-wave sweep: one 8192-cell domain per (alpha0, y) pair, alpha0 in
    32 log-spaced values 0.0022..1 and y in 17 values 0.4..2.0 (544 domains),
    c = 1540, rho = 1000, linear, N = 2.  dx = c / (16 * 20 MHz) (16 points per
    wavelength at the top of the band), CFL 0.2, 24-cell CPML at both ends.
    Broadband source at cell 64: first derivative of a Gaussian with its
    spectral peak at 6 MHz.  Receivers at the measurement cells of
    sweep_receiver_cells (16 per domain, those inside the grid); by default
    the run lasts until the pulse has passed the farthest one."""
    a0 = SWEEP_ALPHA0 if alpha0 is None else np.asarray(alpha0, dtype=np.float64)
    yy = SWEEP_Y if y is None else np.asarray(y, dtype=np.float64)
    A0, Y = np.meshgrid(a0, yy, indexing="ij")
    A0, Y = A0.ravel(), Y.ravel()
    nd = A0.size
    dx = c / (16 * 20e6)
    dt = 0.2 * dx / c
    rc = sweep_receiver_cells(dx, c, src_cell).ravel()
    rc = rc[rc < n_cells - pml]
    if steps is None:
        steps = int(round((int(rc.max()) - src_cell) * dx / c / dt)) + 2000
    sigma = 1.0 / (2.0 * np.pi * 6e6)
    wave = gaussian_derivative(steps, dt, sigma, amplitude=1.0)
    shp = (n_cells, 1, 1)
    return Case(
        name="1d_sweep_%dx%d" % (nd, n_cells), ndim=1, shapes=[shp] * nd, dx=dx, dt=dt, nmech=nmech,
        pml_cells=pml, class_maps=[np.zeros((1, 1, n_cells), np.uint8)] * nd, class_base=list(range(nd)),
        c=np.full(nd, c), rho=np.full(nd, rho), alpha0=A0, y=Y, b_over_a=np.zeros(nd), nonlinear=False,
        src_domain=np.arange(nd, dtype=np.int32), src_cell=np.full(nd, src_cell, np.int64),
        src_wave=np.zeros(nd, np.int32), waves=wave[None, :],
        rec_domain=np.repeat(np.arange(nd, dtype=np.int32), rc.size), rec_cell=np.tile(rc, nd).astype(np.int64),
        n_steps=steps)


def batched_2d(n_shots=64, steps=3000, seed0=4000, nmech=4):
    """Batched 2D shots: square grids with side uniform in 384..1536 (seed
    4000 + s), dx = 50 um, 24-cell CPML, 4 horizontal layers at sorted
    U(0.2, 0.8) L with classes drawn from the 3D tissue ranges (no speed
    perturbation), N = 4, common dt = 0.4 dx / 1650, point source at
    (U[L/4, 3L/4], 28) (3 MHz, 3 cycles), 64 receivers along row 28."""
    dx = 5e-5
    dt = 0.4 * dx / 1650.0
    P = 24
    shapes, maps, base = [], [], []
    cols = {k: [] for k in ("c", "rho", "alpha0", "y", "b_over_a")}
    sd, sc, rd, rc = [], [], [], []
    for s in range(n_shots):
        rng = np.random.default_rng(seed0 + s)
        L = int(rng.integers(384, 1537))
        shp = (L, L, 1)
        bounds = np.sort(rng.uniform(0.2, 0.8, size=3)) * L
        maps.append(layered_labels((1, L, L), bounds.astype(int), axis=1))
        cls = draw_tissue_classes(4, seed0 + 1000 + s)
        for k in cols:
            cols[k].append(cls[k])
        base.append(4 * s)
        shapes.append(shp)
        sx = int(rng.integers(L // 4, 3 * L // 4))
        sd.append(s)
        sc.append(int(linear_index(shp, sx, 28)))
        xs = np.linspace(P + 1, L - P - 2, 64).astype(int)
        rd.extend([s] * 64)
        rc.extend(linear_index(shp, xs, 28).tolist())
    waves = tone_burst(steps, dt, 3e6, 3, amplitude=1e5)[None, :]
    return Case(
        name="2d_batched_%dshots" % n_shots, ndim=2, shapes=shapes, dx=dx, dt=dt, nmech=nmech, pml_cells=P,
        class_maps=maps, class_base=base, c=np.concatenate(cols["c"]), rho=np.concatenate(cols["rho"]),
        alpha0=np.concatenate(cols["alpha0"]), y=np.concatenate(cols["y"]),
        b_over_a=np.concatenate(cols["b_over_a"]), nonlinear=True,
        src_domain=np.array(sd, np.int32), src_cell=np.array(sc, np.int64), src_wave=np.zeros(len(sd), np.int32),
        waves=waves, rec_domain=np.array(rd, np.int32), rec_cell=np.array(rc, np.int64), n_steps=steps)


def adjoint_2d(n=1024, n_shots=16, steps=3000, seed=5, n_rec=128, pml=24):
    """Adjoint workload: n x n (1024 x 1024) with a 24-cell CPML, dx = 50 um,
    6-class smoothed label field (seed 5) with classes from the 3D tissue
    ranges, N = 4, linear; 16 point-source shots evenly spaced on row 28
    (one domain per shot, same medium), 128 receivers on row 28, 3000 steps."""
    dx = 5e-5
    cls = draw_tissue_classes(6, seed)
    dt = 0.4 * dx / 1650.0
    lab = smoothed_label_field((1, n, n), 6, seed, coarse=4, sigma=5.0)
    shp = (n, n, 1)
    xs = np.linspace(pml + 8, n - pml - 9, n_shots).astype(int)
    rx = np.linspace(pml + 1, n - pml - 2, n_rec).astype(int)
    rd = np.repeat(np.arange(n_shots, dtype=np.int32), n_rec)
    rc = np.tile(linear_index(shp, rx, 28), n_shots)
    waves = tone_burst(steps, dt, 2.5e6, 3, amplitude=1e5)[None, :]
    return Case(
        name="2d_adjoint_%dx%d_%dshots" % (n, n, n_shots), ndim=2, shapes=[shp] * n_shots, dx=dx, dt=dt, nmech=4,
        pml_cells=pml, class_maps=[lab] * n_shots, class_base=[0] * n_shots,
        c=cls["c"], rho=cls["rho"], alpha0=cls["alpha0"], y=cls["y"], b_over_a=cls["b_over_a"], nonlinear=False,
        src_domain=np.arange(n_shots, dtype=np.int32), src_cell=linear_index(shp, xs, 28).astype(np.int64),
        src_wave=np.zeros(n_shots, np.int32), waves=waves, rec_domain=rd, rec_cell=rc.astype(np.int64),
        n_steps=steps)
