"""Shared checks of the parity tests (no GPU needed to import)."""
import numpy as np


def one_sided_activations(T, To, v, vo, theta, t_end, dt, tol=1e-4):
    """Voxels activated in one run and not in the other.  Returns the count
    and whether each is explained by the end of the run: the run that fired
    did so during the last step, and the other run's final potential lies
    within tol of the threshold (so FP32 rounding decides which side of
    theta it ends on).  An activation missing earlier than that is a real
    difference."""
    a, b = np.isfinite(T), np.isfinite(To)
    odd = a != b
    if not odd.any():
        return 0, True
    fired = np.where(a, T, To)[odd]
    other_v = np.where(a, vo, v)[odd]
    ok = bool(np.all(fired >= t_end - dt - 1e-9) and np.all(np.abs(other_v - theta) <= tol))
    return int(odd.sum()), ok
