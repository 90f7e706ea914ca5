"""Hand a Case to the product library or to the oracle.

Pure argument passing: each side converts B/A to its nonlinearity coefficient
with its own code.  Imports are lazy so that neither side is loaded unless
asked for; this module is used by the tests, the smoke check and the
benchmark (whose oracle leg is the CPU baseline).
"""
import numpy as np


def to_simulation(case, **kw):
    """Build and configure a product Simulation (HIP library) for the case."""
    from paper_2606_11103_amd.sim import Simulation, beta_from_b_over_a
    sim = Simulation(case.ndim, case.shapes, case.dx, case.dt, case.nmech, case.pml_cells,
                     pml_params=case.pml_params, **kw)
    if case.fd_c_ref > 0 and case.fd_widened:
        sim.set_widened_stencil(case.fd_c_ref)
    elif case.fd_c_ref > 0:
        sim.set_time_space_stencil(case.fd_c_ref)
    beta = beta_from_b_over_a(case.b_over_a) if case.nonlinear else np.zeros(case.n_classes)
    sim.set_media(case.class_maps, case.class_base, case.c, case.rho, beta, case.noise_amp, case.noise_seed)
    sim.set_relaxation_table(case.kappa, case.d, case.alpha)
    if len(case.src_cell):
        sim.set_sources(case.src_domain, case.src_cell, case.src_wave, case.waves)
    if len(case.rec_cell):
        sim.set_receivers(case.rec_domain, case.rec_cell, case.n_steps)
    if case.strength is not None:
        import torch
        flat = np.concatenate([np.asarray(m, np.float32).reshape(-1) for m in case.strength])
        sim.set_strength_map(torch.from_numpy(flat).to(sim.device))
    return sim


def to_oracle(case, domain=0, **kw):
    """Build the FP64 oracle for one domain of the case."""
    from oracle.solver import OracleSim, beta_from_b_over_a
    b = case.class_base[domain]
    nloc = int(case.class_maps[domain].max()) + 1
    sl = slice(b, b + nloc)
    beta = beta_from_b_over_a(case.b_over_a[sl]) if case.nonlinear else np.zeros(nloc)
    pp = case.pml_params or (1e-4, 1e6, 0.0)
    cref = pp[2] if pp[2] > 0 else float(np.max(case.c))
    if case.strength is not None and "a_scale" not in kw:
        kw["a_scale"] = np.asarray(case.strength[domain], np.float64).reshape(-1)
    if case.fd_c_ref > 0 and "fd_c_ref" not in kw:
        kw["fd_c_ref"] = case.fd_c_ref
        kw["off_axis"] = case.fd_widened
    return OracleSim(case.ndim, case.shapes[domain], case.dx, case.dt, case.nmech, case.class_maps[domain],
                     case.c[sl], case.rho[sl], beta, case.kappa[sl], case.d[sl], case.alpha[sl],
                     pml_cells=case.pml_cells, pml_R0=pp[0], pml_f_alpha=pp[1], pml_c_ref=cref,
                     noise_amp=case.noise_amp, noise_seed=case.noise_seed, **kw)


def oracle_traces(case, n_steps=None, energy=False):
    """Run the oracle on every domain; returns traces [n_steps][n_rec] in the
    order of case.rec_cell (FP64)."""
    n = case.n_steps if n_steps is None else n_steps
    out = np.zeros((n, len(case.rec_cell)))
    for d in range(len(case.shapes)):
        sim = to_oracle(case, d)
        sm = case.src_domain == d
        rm = np.nonzero(case.rec_domain == d)[0]
        waves = case.waves.astype(np.float64)[case.src_wave[sm]]
        rec, _ = sim.run(n, case.src_cell[sm], waves, case.rec_cell[rm])
        out[:, rm] = rec
    return out


def to_oracle_crop(case, lo, hi, domain=0):
    """Oracle for the box [lo, hi) (x, y, z cell bounds) of one domain: class
    map, speed perturbation (keyed by the full-domain index) and CPML
    profiles of the full axes restricted to the box.  Valid while the field
    is zero outside the box (e.g. a few steps after the sources start)."""
    from oracle.solver import OracleSim, beta_from_b_over_a
    nx, ny, nz = case.shapes[domain]
    lo = [int(v) for v in lo]
    hi = [int(v) for v in hi]
    cm = case.class_maps[domain][lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                             indexing="ij")
    full_index = (zz.astype(np.int64) * ny + yy) * nx + xx
    b = case.class_base[domain]
    nloc = int(case.class_maps[domain].max()) + 1
    sl = slice(b, b + nloc)
    beta = beta_from_b_over_a(case.b_over_a[sl]) if case.nonlinear else np.zeros(nloc)
    pp = case.pml_params or (1e-4, 1e6, 0.0)
    cref = pp[2] if pp[2] > 0 else float(np.max(case.c))
    shape = (hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
    axis_full = [(nx, lo[0]), (ny, lo[1]), (nz, lo[2])]
    return OracleSim(case.ndim, shape, case.dx, case.dt, case.nmech, cm, case.c[sl], case.rho[sl], beta,
                     case.kappa[sl], case.d[sl], case.alpha[sl], pml_cells=case.pml_cells, pml_R0=pp[0],
                     pml_f_alpha=pp[1], pml_c_ref=cref, noise_amp=case.noise_amp, noise_seed=case.noise_seed,
                     noise_index=full_index, axis_full=axis_full)
