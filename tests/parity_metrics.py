"""Trace comparison used by every GPU-vs-oracle parity test.

Two figures, both in FP64 over the receiver traces [steps x receivers]:
* the global relative L2 error, ||got - ref|| / ||ref||;
* the worst relative L2 error of a single reached receiver, so that an error
  confined to weak receivers (inside a CPML slab, behind a strong
  attenuator, in a late tail) is not diluted by the strong ones.  A receiver
  counts as reached when its oracle trace peaks at >= REACH of the strongest
  receiver's peak; weaker ones, where the field is numerically zero or only
  the stencil's exponentially small precursor has arrived, carry no
  information about the arithmetic.
The bar for both is the accuracy target of the workload: 1e-4.
"""
import numpy as np

TOL = 1e-4
REACH = 1e-3


def trace_errors(got, ref, reach=REACH):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    glob = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    peak = np.abs(ref).max(axis=0)
    reached = peak >= reach * peak.max()
    per = np.linalg.norm((got - ref)[:, reached], axis=0) / np.linalg.norm(ref[:, reached], axis=0)
    return glob, float(per.max()), int(reached.sum())


def check_traces(got, ref, tol=TOL):
    """Assert both figures; returns (global, worst receiver, reached count)."""
    got = np.asarray(got, np.float64)
    assert np.all(np.isfinite(got))
    assert np.abs(ref).max() > 0
    glob, worst, n = trace_errors(got, ref)
    assert glob <= tol, "global rel L2 %.3e" % glob
    assert worst <= tol, "worst reached receiver rel L2 %.3e" % worst
    return glob, worst, n
