"""Comparison of two simulation states on what is state: g and the fronts
everywhere, f in the liquid cells only.  The f of a solid cell is never read
(a liquid neighbour bounces back from it, a melting cell is refilled with
the rest state) and the library does not write it, so it holds whatever its
buffer held before."""
import numpy as np


def liquid_mask(s, heating="y0"):
    """[z][y][x] mask of the liquid cells for fronts s (column layout)."""
    n = s.shape[0]
    a = np.arange(n) + 0.5
    if heating == "y0":  # melt axis y, s[z][x]
        return a[None, :, None] < s[:, None, :]
    return a[:, None, None] < s[None, :, :]  # melt axis z, s[y][x]


def states_equal(pa, pb, heating="y0"):
    """Bitwise equality of two (f, g, s) states on their live parts."""
    fa, ga, sa = pa
    fb, gb, sb = pb
    if not (np.array_equal(ga, gb) and np.array_equal(sa, sb)):
        return False
    if fa is None or fb is None:
        return fa is None and fb is None
    m = liquid_mask(sa, heating)
    return bool(np.array_equal(fa[:, m], fb[:, m]))
