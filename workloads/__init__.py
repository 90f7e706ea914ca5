"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws media, source waveforms and source/receiver geometry.  It
holds none of the method's arithmetic: no stencil, no relaxation coefficient,
no fit, no unit conversion of the attenuation law.  Both the product path and
the FP64 oracle receive exactly the arrays produced here (waveforms are
rounded to FP32 once, and both sides read those values).

The recipes mirror the paper's workloads (Sec. 4 and Sec. 5):
Gaussian-modulated sinusoidal pulses (Sec. 4.1), plane-wave line sources at the
top of the domain (Sec. 4.1), two-layer media (Sec. 4.4), tissue parameters in
the ranges of Sec. 3 / Table 3, and a seeded smooth random label field standing
in for the segmented abdomen volume of Sec. 4.5, which is not available.
"""
import math

import numpy as np

TISSUE_RANGES = dict(c=(1400.0, 1650.0), rho=(900.0, 1100.0), alpha0=(0.0022, 1.0),
                     y=(0.4, 2.0), b_over_a=(5.0, 10.0))


# ------------------------------------------------------------------ pulses --
def tone_burst(n_t, dt, f0, n_cycles, amplitude=1.0, delay=0.0):
    """Gaussian-windowed sine sampled at t_s = (s + 1) dt, s = 0..n_t-1:
    A sin(2 pi f0 (t - t0)) exp(-((t - t0)/sigma)^2), sigma = n_cycles/(2 f0),
    t0 = 4 sigma + delay.  Returned as float32 (the values both sides use)."""
    t = (np.arange(n_t, dtype=np.float64) + 1.0) * dt
    sigma = n_cycles / (2.0 * f0)
    t0 = 4.0 * sigma + delay
    w = amplitude * np.sin(2.0 * np.pi * f0 * (t - t0)) * np.exp(-((t - t0) / sigma) ** 2)
    return w.astype(np.float32)


def gaussian_derivative(n_t, dt, sigma, amplitude=1.0, t0=None):
    """Broadband first-derivative-of-Gaussian pulse -u exp(-u^2/2),
    u = (t - t0)/sigma: amplitude spectrum f exp(-(2 pi f sigma)^2 / 2), peak
    at 1/(2 pi sigma); sampled at t_s = (s + 1) dt, float32."""
    t = (np.arange(n_t, dtype=np.float64) + 1.0) * dt
    t0 = 5.0 * sigma if t0 is None else t0
    u = (t - t0) / sigma
    w = -amplitude * u * np.exp(-0.5 * u * u) * math.exp(0.5)
    return w.astype(np.float32)


# ------------------------------------------------------------------- media --
def draw_tissue_classes(n, seed, ranges=TISSUE_RANGES):
    """n tissue classes: c, rho, y and B/A uniform, alpha0 log-uniform."""
    rng = np.random.default_rng(seed)
    lo, hi = ranges["alpha0"]
    return dict(
        c=rng.uniform(*ranges["c"], size=n),
        rho=rng.uniform(*ranges["rho"], size=n),
        alpha0=10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=n),
        y=rng.uniform(*ranges["y"], size=n),
        b_over_a=rng.uniform(*ranges["b_over_a"], size=n),
    )


def smoothed_label_field(shape_zyx, n_classes, seed, coarse=4, sigma=5.0):
    """Label field = argmax over n_classes iid N(0,1) fields drawn at 1/coarse
    resolution, Gaussian-smoothed (sigma in coarse cells), then upsampled by
    nearest neighbour.  Ties go to the lowest class index.  uint8."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    cshape = tuple(max(1, -(-s // coarse)) for s in shape_zyx)
    best = None
    lab = np.zeros(cshape, dtype=np.uint8)
    for k in range(n_classes):
        f = gaussian_filter(rng.standard_normal(cshape).astype(np.float32), sigma, mode="wrap")
        if best is None:
            best = f
        else:
            m = f > best
            lab[m] = k
            best = np.where(m, f, best)
    for ax, s in enumerate(shape_zyx):
        lab = np.repeat(lab, coarse, axis=ax).take(np.arange(s), axis=ax)
    return np.ascontiguousarray(lab)


def smooth_unit_field(shape_zyx, seed, lo=0.2, hi=1.0, sigma=3.0):
    """Smooth random field with values in [lo, hi]: an iid N(0, 1) field,
    Gaussian-smoothed (sigma cells), rescaled to its own min..max and mapped
    onto [lo, hi]; float32 (the values both sides read)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    f = gaussian_filter(rng.standard_normal(shape_zyx), sigma, mode="wrap")
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return np.ascontiguousarray((lo + (hi - lo) * f).astype(np.float32))


def layered_labels(shape_zyx, boundaries, axis):
    """Piecewise-constant labels along one axis: class k between
    boundaries[k-1] and boundaries[k] (cell indices)."""
    n = shape_zyx[axis]
    lab1 = np.zeros(n, dtype=np.uint8)
    for k, b in enumerate(sorted(boundaries)):
        lab1[int(b):] = k + 1
    sh = [1] * len(shape_zyx)
    sh[axis] = n
    return np.ascontiguousarray(np.broadcast_to(lab1.reshape(sh), shape_zyx).astype(np.uint8))


def linear_index(shape_xyz, x, y=0, z=0):
    nx, ny, _ = shape_xyz
    return (np.asarray(z, dtype=np.int64) * ny + np.asarray(y, dtype=np.int64)) * nx + np.asarray(x, dtype=np.int64)
