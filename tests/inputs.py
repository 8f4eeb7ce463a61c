"""Seeded synthetic inputs shared by the oracle side and the GPU side of the
tests.  Holds no arithmetic of the method: only random numbers of the right
shapes and ranges."""
import numpy as np


def random_state(n, seed, flow=True, front=(0.0, None)):
    """Populations with random positive values (f in [0.02, 0.06], g in
    [0, 0.2]) and a rough front: independent uniform heights per column in
    [front[0], front[1]] (default: the whole box)."""
    rng = np.random.default_rng(seed)
    lo, hi = front[0], (n if front[1] is None else front[1])
    f = rng.uniform(0.02, 0.06, size=(19, n, n, n)) if flow else None
    g = rng.uniform(0.0, 0.2, size=(7, n, n, n))
    s = lo + (hi - lo) * rng.random((n, n))
    return f, g, s


def hot_wall_field(n, seed=0, mean=1.0, spread=0.1):
    """Hot-wall temperature per column: mean + spread * N(0, 1)."""
    rng = np.random.default_rng(seed)
    return mean + spread * rng.standard_normal((n, n))
