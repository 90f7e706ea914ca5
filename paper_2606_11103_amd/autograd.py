"""torch.autograd.Function around the checkpointed HIP adjoint.

traces = FDTDFunction.apply(c_map, alpha0_map, problem)

* c_map, alpha0_map: per-voxel sound speed (m/s) and attenuation coefficient
  alpha0 (dB/(MHz^y cm)), torch tensors over all cells of all domains in the
  unpadded layout (domains concatenated, each in its own linear order).
* problem: a Problem (below) with the tissue labels and, per label, the
  reference class (c, rho, alpha0, y, relaxation table) plus grid, sources and
  receivers.

The forward run groups voxels into classes by (label, c, alpha0); a class
keeps its label's kappa and alpha and scales the label's d by
alpha0 / alpha0_label (Sec. 2.1 parameters; d-scaling keeps the relaxation
times and scales the relaxation strength).  At most 256 distinct classes per
domain are allowed, so continuous maps must be quantised first, and every
alpha0 must be > 0.  The backward pass feeds dJ/d traces to the HIP adjoint
(fw_adjoint), which returns dJ/dc(x) and dJ/dalpha0(x) per voxel; this
module only marshals arrays.  Linear media only (beta = 0), as the adjoint
is.
"""
import dataclasses
from typing import List, Optional

import numpy as np
import torch

from .sim import Simulation


@dataclasses.dataclass
class Problem:
    ndim: int
    shapes: List[tuple]
    dx: float
    dt: float
    nmech: int
    pml_cells: int
    labels: List[np.ndarray]          # uint8 per domain, label index into the tables below
    rho: np.ndarray                   # [n_labels]
    alpha0_ref: np.ndarray            # [n_labels]
    kappa: np.ndarray                 # [n_labels][2]
    d: np.ndarray                     # [n_labels][2][N]
    alpha: np.ndarray                 # [n_labels][2][N]
    src_domain: np.ndarray
    src_cell: np.ndarray
    src_wave: np.ndarray
    waves: np.ndarray
    rec_domain: np.ndarray
    rec_cell: np.ndarray
    n_steps: int
    ckpt_every: int = 55
    noise_amp: float = 0.0
    noise_seed: int = 0
    pml_params: Optional[tuple] = None


def _classes(problem, c, a0):
    """Group voxels into classes by (label, c, alpha0) per domain."""
    maps, base, cls_c, cls_rho, cls_k, cls_d, cls_al, cls_a0 = [], [], [], [], [], [], [], []
    pos = 0
    nb = 0
    for dom, shp in enumerate(problem.shapes):
        n = int(np.prod(shp))
        lab = np.asarray(problem.labels[dom]).reshape(-1).astype(np.int64)
        key = np.stack([lab.astype(np.float64), c[pos:pos + n], a0[pos:pos + n]], axis=1)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        if len(uniq) > 256:
            raise ValueError("domain %d has %d distinct (label, c, alpha0) classes; at most 256 are supported "
                             "(quantise the maps)" % (dom, len(uniq)))
        maps.append(inv.reshape(np.asarray(problem.labels[dom]).shape).astype(np.uint8))
        base.append(nb)
        for lbl, cc, aa in uniq:
            L = int(lbl)
            cls_c.append(cc)
            cls_rho.append(problem.rho[L])
            cls_k.append(problem.kappa[L])
            cls_d.append(problem.d[L] * (aa / problem.alpha0_ref[L]))
            cls_al.append(problem.alpha[L])
            cls_a0.append(aa)
        nb += len(uniq)
        pos += n
    return (maps, base, np.array(cls_c), np.array(cls_rho), np.array(cls_k), np.array(cls_d), np.array(cls_al),
            np.array(cls_a0))


class FDTDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c_map, alpha0_map, problem):
        c = c_map.detach().double().cpu().numpy().reshape(-1)
        a0 = alpha0_map.detach().double().cpu().numpy().reshape(-1)
        if not np.all(a0 > 0):
            raise ValueError("alpha0 must be > 0 in every voxel (the relaxation strengths scale with it)")
        maps, base, cc, rho, kap, d, al, ca0 = _classes(problem, c, a0)
        sim = Simulation(problem.ndim, problem.shapes, problem.dx, problem.dt, problem.nmech, problem.pml_cells,
                         pml_params=problem.pml_params)
        sim.set_media(maps, base, cc, rho, np.zeros(len(cc)), problem.noise_amp, problem.noise_seed)
        sim.set_relaxation_table(kap, d, al)
        sim.set_class_alpha0(ca0)
        sim.set_sources(problem.src_domain, problem.src_cell, problem.src_wave, problem.waves)
        sim.set_receivers(problem.rec_domain, problem.rec_cell, problem.n_steps)
        work = sim.adjoint_workspace(problem.n_steps, problem.ckpt_every)
        sim.forward_checkpointed(problem.n_steps, problem.ckpt_every, work)
        traces = sim.read_receivers_device()
        ctx.sim, ctx.work, ctx.problem = sim, work, problem
        ctx.in_device = c_map.device
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        sim, work, problem = ctx.sim, ctx.work, ctx.problem
        grad_c, grad_a0 = sim.adjoint(problem.n_steps, problem.ckpt_every, work, grad_traces.detach().float())
        ctx.sim = ctx.work = None
        return grad_c.to(ctx.in_device), grad_a0.to(ctx.in_device), None


def simulate(c_map, alpha0_map, problem):
    """Differentiable receiver traces [n_steps][n_rec] (device tensor)."""
    return FDTDFunction.apply(c_map, alpha0_map, problem)
