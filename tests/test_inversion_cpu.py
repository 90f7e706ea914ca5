"""Host logic of the label-wise inversion: the scaled quasi-Newton descent
with its quadratic line search, on closed-form misfits (no GPU)."""
import numpy as np

from paper_2606_11103_amd.inversion import descend


def test_descent_reaches_the_minimum_of_a_quadratic():
    xs = np.array([1480.0, 1575.0, 1520.0])
    w = np.array([1.0, 4.0, 0.25])

    def ev(x, want_grad):
        r = x - xs
        return float(np.sum(w * r * r)), (2 * w * r if want_grad else None)

    x, J, steps = descend(ev, xs + np.array([20.0, -15.0, 30.0]), np.full(3, 10.0), iters=40)
    assert all(b < a for a, b in zip(J, J[1:]))                 # every accepted step lowers J
    assert np.max(np.abs(x - xs)) < 0.5 and J[-1] < 1e-3 * J[0]


def test_groups_are_scaled_separately():
    """Two groups of very different units: each moves by its own scale."""
    xs = np.array([1500.0, 0.5])

    def ev(x, want_grad):
        r = x - xs
        return float(r[0] ** 2 + 1e6 * r[1] ** 2), (np.array([2 * r[0], 2e6 * r[1]]) if want_grad else None)

    x, J, _ = descend(ev, np.array([1510.0, 0.6]), np.array([4.0, 0.02]), iters=30,
                      groups=[np.array([0]), np.array([1])])
    assert abs(x[0] - 1500.0) < 0.2 and abs(x[1] - 0.5) < 2e-3


def test_descent_stops_when_no_step_lowers_the_misfit():
    def ev(x, want_grad):                                        # minimum at the start point
        return float(np.sum(x * x)), (2 * x if want_grad else None)

    x, J, steps = descend(ev, np.zeros(2) + 1e-9, np.full(2, 1.0), iters=5, max_halvings=3)
    assert len(J) == 1 and steps == [] and np.allclose(x, 1e-9)


def test_correlated_parameters_converge_quickly():
    """An ill-conditioned quadratic with strongly coupled parameters (a valley
    across the scaled axes): BFGS reaches it in a few iterations."""
    xs = np.array([1500.0, 0.5, 1600.0, 0.9])
    Q, _ = np.linalg.qr(np.array([[1.0, 0.9, 0.2, 0.0], [0.3, 1.0, 0.8, 0.1], [0.0, 0.4, 1.0, 0.7],
                                  [0.2, 0.0, 0.5, 1.0]]))
    A = Q @ np.diag([5.0, 1.0, 0.05, 0.0005]) @ Q.T          # condition number 1e4
    sc = np.array([5.0, 0.05, 5.0, 0.05])

    def ev(x, want_grad):
        r = (x - xs) / sc
        return float(r @ A @ r), ((2 * A @ r) / sc if want_grad else None)

    x0 = xs + np.array([12.0, 0.12, -9.0, -0.2])
    x, J, _ = descend(ev, x0, sc, iters=25, groups=[np.array([0, 2]), np.array([1, 3])])
    assert J[-1] < 1e-10 * J[0] and len(J) <= 26
    assert np.max(np.abs((x - xs) / sc)) < 1e-3
