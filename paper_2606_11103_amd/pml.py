"""Two-stage absorbing layer and the 2D reflection protocol.

Sec. 4.3 measures the reflection of the absorbing boundary with a plane wave
from the top of a D = 5 wavelength deep, W = 20 wavelength wide domain onto
the bottom layer, at 1 MHz; Sec. 4.6 and Sec. 5.4/5.5 compare the adaptive
two-stage layer (a transition region of L_T = 3 wavelengths before a C-PML
of L_B = 3 wavelengths, relaxation parameters matching the local tissue)
with a homogeneous layer (parameters of one fixed tissue, (alpha0, y) =
(0.5, 1.0)) with and without the transition region, and report that without
it the relaxation parameters are ramped inside the C-PML instead.

The paper does not print the layer's equations (they are in its companion
paper).  Reading taken here: across the transition region the tissue's
relaxation is ramped down to the lossless medium, so that the C-PML behind it
absorbs in a medium without memory variables, where an additive and a
composed C-PML stretch coincide.  At depth fraction s in (0, 1) of the ramp
the weight is w = sin^2(pi s / 2) and the class gets
    1/kappa_w = 1 + (1 - w) (1/kappa - 1),  d_w = (1 - w) d,  alpha unchanged,
per operator and mechanism (one class per cell row of the ramp).  Designs:
    "composed"         the library's single-stage layer: the tissue continues
                       into the C-PML, whose stretch multiplies the tissue's;
    "two_stage"        local tissue, ramped to lossless across L_T, then the
                       C-PML in the lossless medium;
    "homog_two_stage"  the absorbing region (transition and C-PML) holds the
                       fixed reference tissue instead of the local one,
                       ramped to lossless across L_T;
    "homog_one_stage"  no transition region: the reference tissue ramped to
                       lossless across the C-PML itself.
Only the bottom boundary follows the design; the top and side layers are the
library's (their echoes are the same in the measurement and reference runs
and cancel in the difference).
"""
import numpy as np

from . import relax

DESIGNS = ("composed", "two_stage", "homog_two_stage", "homog_one_stage")


def ramp_weights(n):
    """w of the n ramp rows, w = sin^2(pi s / 2) at s = (i + 1/2) / n."""
    s = (np.arange(n, dtype=np.float64) + 0.5) / n
    return np.sin(0.5 * np.pi * s) ** 2


def ramped(kappa, d, alpha, w):
    """One tissue table [2], [2][N], [2][N] ramped towards the lossless
    medium by weight w (0: the tissue, 1: lossless)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    ik = 1.0 + (1.0 - w) * (1.0 / kappa - 1.0)
    return 1.0 / ik, (1.0 - w) * np.asarray(d, dtype=np.float64), np.asarray(alpha, dtype=np.float64).copy()


def bottom_layer_tables(kappa, d, alpha, design, n_trans, n_pml, ref=None):
    """Class tables of one domain whose bottom boundary follows design:
    class 0 the interior tissue; rows of the transition region, then rows of
    the C-PML slab, each get a class.  Returns (kappa [C][2], d [C][2][N],
    alpha [C][2][N], row_class (per boundary row, top to bottom: n_trans rows
    of transition then n_pml rows of the slab))."""
    if design not in DESIGNS:
        raise ValueError("unknown layer design %r" % design)
    tissue = (np.asarray(kappa, np.float64), np.asarray(d, np.float64), np.asarray(alpha, np.float64))
    lossless = ramped(*tissue, 1.0)
    if design == "composed":
        tabs = [tissue]
        rows = [0] * (n_trans + n_pml)
    else:
        src = tissue if design == "two_stage" else tuple(np.asarray(x, np.float64) for x in ref)
        if design == "homog_one_stage":
            ramp_rows, slab_rows = n_pml, 0
            pre = [0] * n_trans            # no transition: interior tissue down to the slab
        else:
            ramp_rows, slab_rows = n_trans, n_pml
            pre = []
        tabs = [tissue] + [ramped(*src, w) for w in ramp_weights(ramp_rows)] + [lossless]
        rows = pre + list(range(1, ramp_rows + 1)) + [ramp_rows + 1] * slab_rows
    k = np.array([t[0] for t in tabs])
    dd = np.array([t[1] for t in tabs])
    al = np.array([t[2] for t in tabs])
    return k, dd, al, np.array(rows, dtype=np.int64)


def reflection_2d(kappa, d, alpha, design="composed", ref=None, c=1540.0, rho=1000.0, f0=1e6, ppw=16, cfl=0.2,
                  trans_wavelengths=3.0, pml_wavelengths=3.0, depth_wavelengths=5.0, width_wavelengths=20.0,
                  n_cycles=3, step_match=True, return_traces=False):
    """Reflection of the bottom boundary in dB for each table (kappa [T][2],
    d and alpha [T][2][N]), Sec. 4.3 protocol in 2D: a plane-wave line
    source across the domain below the top layer, D below it the bottom
    boundary (transition region, if any, then the C-PML), a receiver on the
    centre column at 0.8 D, a 1 MHz Gaussian-modulated pulse; 16 points per
    wavelength and CFL 0.2 (Sec. 3.3).  Each table runs in two domains of
    one batched 2D launch: one ending in the bottom boundary and one deep
    enough that nothing returns from its bottom within the window; the
    reflected wave is the difference of the two receiver traces,
    R = 20 log10(max|difference| / max|incident|).  ref is the reference
    tissue table (kappa [2], d [2][N], alpha [2][N]) of the homogeneous
    designs.  With step_match, tables (and ref) are relax.step_matched to
    the run's time step first."""
    from .sim import Simulation
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    n_tab, nmech = kappa.shape[0], d.shape[2]
    lam = c / f0
    dx = lam / ppw
    dt = cfl * dx / c
    if design.startswith("homog") and ref is None:
        raise ValueError("the homogeneous designs need the reference tissue table")
    if step_match:
        kappa, d, alpha = relax.step_matched(kappa, d, alpha, dt)
        if ref is not None:
            k_r, d_r, a_r = relax.step_matched(np.asarray(ref[0])[None], np.asarray(ref[1])[None],
                                               np.asarray(ref[2])[None], dt)
            ref = (k_r[0], d_r[0], a_r[0])
    P = int(round(pml_wavelengths * ppw))
    LT = int(round(trans_wavelengths * ppw)) if design != "composed" else 0
    if design == "homog_one_stage":
        LT = 0
    D = int(round(depth_wavelengths * ppw))
    W = int(round(width_wavelengths * ppw))
    nx = W + 2 * P
    src = P + 4
    rec = src + int(round(0.8 * D))
    sigma = n_cycles / (2.0 * f0)
    travel = (2 * (src + D) - src - rec) * dx / c
    n_steps = int(np.ceil((travel + 10.0 * sigma) / dt))
    ny_short = src + D + LT + P
    ny_long = ny_short + int(np.ceil(n_steps * cfl / 2.0)) + P + 8
    shapes, maps, base = [], [], []
    ks, ds, als = [], [], []
    nb = 0
    for j in range(n_tab):
        k_j, d_j, a_j, rows = bottom_layer_tables(kappa[j], d[j], alpha[j], design, LT, P, ref)
        lab = np.zeros((1, ny_short, nx), np.uint8)
        lab[0, ny_short - LT - P:, :] = rows.astype(np.uint8)[:, None]
        shapes += [(nx, ny_short, 1), (nx, ny_long, 1)]
        maps += [lab, np.zeros((1, ny_long, nx), np.uint8)]
        base += [nb, nb]
        ks.append(k_j)
        ds.append(d_j)
        als.append(a_j)
        nb += k_j.shape[0]
    ks, ds, als = np.concatenate(ks), np.concatenate(ds), np.concatenate(als)
    nd = 2 * n_tab
    t = (np.arange(n_steps) + 1.0) * dt - 4.0 * sigma
    wave = (np.sin(2.0 * np.pi * f0 * t) * np.exp(-(t / sigma) ** 2)).astype(np.float32)
    src_dom = np.repeat(np.arange(nd), nx)
    src_cell = np.tile(src * nx + np.arange(nx), nd)
    sim = Simulation(2, shapes, dx, dt, nmech, P, pml_params=(1e-4, 1e6, c))
    try:
        sim.set_media(maps, base, np.full(nb, c), np.full(nb, rho), np.zeros(nb))
        sim.set_relaxation_table(ks, ds, als)
        sim.set_sources(src_dom, src_cell, np.zeros(src_dom.size), wave[None, :])
        sim.set_receivers(np.arange(nd), np.full(nd, rec * nx + nx // 2), n_steps)
        sim.step(n_steps)
        tr = sim.read_receivers().astype(np.float64)
    finally:
        sim.close()
    short, long_ = tr[:, 0::2], tr[:, 1::2]
    refl = np.abs(short - long_).max(axis=0)
    inc = np.abs(long_).max(axis=0)
    R = 20.0 * np.log10(np.maximum(refl, 1e-300) / inc)
    if return_traces:
        return R, dict(short=short, long=long_, dx=dx, dt=dt, nx=nx, ny=(ny_short, ny_long), src=src, rec=rec,
                       P=P, LT=LT, n_steps=n_steps, wave=wave, tables=(ks, ds, als), base=base)
    return R


def stats(R, bar=-50.0):
    """Median, worst and the fraction below bar of finite reflections, plus
    the count of non-finite (diverged) runs."""
    R = np.asarray(R, dtype=np.float64)
    ok = np.isfinite(R)
    return dict(n=int(R.size), median=float(np.median(R[ok])) if ok.any() else None,
                worst=float(R[ok].max()) if ok.any() else None,
                frac_below=float(np.mean(R[ok] < bar)) if ok.any() else 0.0, diverged=int((~ok).sum()))
