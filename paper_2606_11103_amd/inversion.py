"""Label-wise inversion of sound speed (and optionally attenuation) from
receiver traces, on top of the differentiable forward run (autograd.simulate,
whose backward pass is the checkpointed HIP adjoint).

Parameters are one c and one alpha0 per tissue label. An iteration runs one
checkpointed forward and one adjoint sweep and sums the per-voxel gradients
over each label. Steps are quasi-Newton (BFGS) in coordinates scaled by
`step_c` m/s and `step_a` times alpha0; the first moves the label with the
largest scaled gradient by one scale unit. A quadratic line search (with
halving) picks the step on the misfit
    J = 1/2 dt sum_n sum_r (trace - observed)^2;
the loop stops when no step lowers it.
"""
import dataclasses
from typing import Callable, List, Optional, Tuple

import numpy as np
import torch

from .autograd import simulate


@dataclasses.dataclass
class InversionResult:
    c: np.ndarray                 # per label, final
    alpha0: np.ndarray            # per label, final
    misfits: List[float]          # J at the start and after each accepted step
    steps: List[float]            # accepted step, as a fraction of the scaled direction


def misfit(traces, observed, dt):
    return 0.5 * dt * ((traces.double() - observed.double()) ** 2).sum()


def descend(evaluate: Callable[[np.ndarray, bool], Tuple[float, Optional[np.ndarray]]], x0: np.ndarray,
            scale: np.ndarray, iters: int, groups: Optional[List[np.ndarray]] = None, max_halvings: int = 6):
    """Quasi-Newton (BFGS) descent in scaled coordinates u = x / scale, with a
    quadratic line search.

    evaluate(x, want_grad) -> (J, dJ/dx or None).  The first direction (and
    any that does not descend) moves each group of components (one group by
    default) by -g_u / max|g_u| in scaled units, so the component with the
    group's largest gradient moves by its full scale; later directions are
    -H g_u with the BFGS inverse-Hessian estimate H.  Along a direction, J is
    fitted by the parabola through J(0), the slope and J(t); its minimiser is
    evaluated too and the lower point is taken if it lowers J, else t is
    halved.  Returns (x, misfits, steps)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    scale = np.asarray(scale, dtype=np.float64)
    groups = groups if groups is not None else [np.arange(len(x))]
    J, g = evaluate(x, True)
    misfits, steps = [J], []
    H = None
    for _ in range(iters):
        if not np.isfinite(J):
            break
        gu = g * scale
        d = -H @ gu if H is not None else None
        if d is None or not float(np.dot(gu, d)) < 0.0:
            d = np.zeros_like(x)
            for idx in groups:
                gmax = float(np.max(np.abs(gu[idx])))
                if gmax > 0.0:
                    d[idx] = -gu[idx] / gmax
            H = None
        slope = float(np.dot(gu, d))
        if not slope < 0.0:
            break
        t, best = 1.0, None
        for _ in range(max_halvings + 1):
            Jt, _ = evaluate(x + t * d * scale, False)
            cands = [(Jt, t)] if np.isfinite(Jt) else []
            curv = (Jt - J - slope * t) / (t * t) if np.isfinite(Jt) else 0.0
            if curv > 0.0:
                ts = min(t, max(t / 16.0, -slope / (2.0 * curv)))
                if ts != t:
                    Js, _ = evaluate(x + ts * d * scale, False)
                    if np.isfinite(Js):
                        cands.append((Js, ts))
            if cands:
                Jb, tb = min(cands)
                if Jb < J:
                    best = tb
                    break
            t *= 0.5
        if best is None:
            break
        su = best * d
        x = x + su * scale
        J, g_new = evaluate(x, True)
        yu = (g_new - g) * scale
        g = g_new
        sy = float(np.dot(su, yu))
        if sy > 1e-12 * float(np.dot(su, su)) * max(float(np.dot(yu, yu)), 1e-300) ** 0.5:
            if H is None:
                H = np.eye(len(x)) * (sy / float(np.dot(yu, yu)))
            rho = 1.0 / sy
            I = np.eye(len(x))
            H = (I - rho * np.outer(su, yu)) @ H @ (I - rho * np.outer(yu, su)) + rho * np.outer(su, su)
        misfits.append(J)
        steps.append(best)
    return x, misfits, steps


def invert_labels(problem, observed, c0, alpha0_0, iters=6, invert_alpha=False, step_c=10.0, step_a=0.1,
                  max_halvings=6) -> InversionResult:
    """Recover per-label c (and alpha0 with invert_alpha) from `observed`
    traces [n_steps][n_rec] of `problem` (an autograd.Problem), starting from
    c0, alpha0_0 (per label)."""
    flat = torch.as_tensor(np.concatenate([np.asarray(l).reshape(-1) for l in problem.labels]).astype(np.int64))
    obs = torch.as_tensor(observed).double()
    n_lab = len(c0)
    a_fixed = np.asarray(alpha0_0, dtype=np.float64)

    def split(x):
        return (x[:n_lab], x[n_lab:]) if invert_alpha else (x, a_fixed)

    def evaluate(x, want_grad):
        c, a = split(x)
        ct = torch.tensor(c, dtype=torch.float64, requires_grad=want_grad)
        at = torch.tensor(a, dtype=torch.float64, requires_grad=want_grad and invert_alpha)
        if not want_grad:
            with torch.no_grad():
                return float(misfit(simulate(ct[flat], at[flat], problem), obs.to("cuda"), problem.dt)), None
        J = misfit(simulate(ct[flat], at[flat], problem), obs.to("cuda"), problem.dt)
        J.backward()
        g = ct.grad.numpy().copy()
        if invert_alpha:
            g = np.concatenate([g, at.grad.numpy()])
        return float(J.detach()), g

    x0 = np.concatenate([c0, alpha0_0]) if invert_alpha else np.asarray(c0, dtype=np.float64)
    scale = np.full(n_lab, float(step_c))
    groups = [np.arange(n_lab)]
    if invert_alpha:
        scale = np.concatenate([scale, float(step_a) * np.asarray(alpha0_0, dtype=np.float64)])
        groups.append(np.arange(n_lab, 2 * n_lab))
    x, misfits, steps = descend(evaluate, x0, scale, iters, groups, max_halvings)
    c, a = split(x)
    return InversionResult(c=np.asarray(c), alpha0=np.asarray(a), misfits=misfits, steps=steps)
