"""Closed-form steady state of pure conduction on the D3Q7 lattice in a
linear temperature field that equals T_m on a tilted plane front.

With the flow frozen, collision conserves T, relaxes the first moments at
rate q_j and leaves the even moments of a field w_q (T + c e_q . grad T) at
equilibrium.  The populations
    g*_q(x) = w_q [T(x) + (1 - 1/q_j) e_q . grad T]
are therefore reproduced by one step wherever the streamed populations equal
the pull from the linear field (section 2, Eq. (4) and Eq. (5)).  At the
front, both branches of the interpolated anti-bounce-back of T = T_m return
that pull exactly for a plane front, and so does the anti-bounce-back of a
hot wall held at the field's value on the wall plane.  Used by the oracle's
pins and by the GPU parity tests; it holds no code of either side.
"""
import numpy as np

T_M = 0.3
GRAD = -0.05  # dT / d(melt coordinate): the liquid below the front is warmer
SLOPE_X, SLOPE_O = -0.31, 0.17  # ds/dx and ds/do of the plane front


def plane_front(n):
    """Front height per column [o][x] (o: z for heating 0, y for heating 1)."""
    c = np.arange(n) + 0.5 - 0.5 * n
    return 0.5 * n + 0.2 + SLOPE_X * c[None, :] + SLOPE_O * c[:, None]


def fixed_point_state(n, heating, q_j, w7, e7):
    """(g*, s, th): the steady post-collision populations of the linear field
    T = T_m + G (h - s(x, o)) in both phases ([q][z][y][x]), the plane front
    and the hot-wall temperatures that continue the field to the wall plane
    h = 0."""
    s = plane_front(n)
    h = np.arange(n) + 0.5
    if heating == 0:  # melt axis y, columns [z][x]
        T = T_M + GRAD * (h[None, :, None] - s[:, None, :])
        grad = np.array([-GRAD * SLOPE_X, GRAD, -GRAD * SLOPE_O])
    else:  # melt axis z, columns [y][x]
        T = T_M + GRAD * (h[:, None, None] - s[None, :, :])
        grad = np.array([-GRAD * SLOPE_X, -GRAD * SLOPE_O, GRAD])
    B = 1.0 - 1.0 / q_j
    g = np.stack([w7[q] * (T + B * float(np.dot(e7[q], grad))) for q in range(7)])
    th = T_M + GRAD * (0.0 - s)
    return g, s, th


def interior(n, heating):
    """Cells whose links stay off the adiabatic lateral walls and the far
    wall (the hot wall at melt index 0 is exact: its value continues the
    field).  Boolean [z][y][x]."""
    m = np.zeros((n, n, n), dtype=bool)
    if heating == 0:
        m[1:n - 1, 0:n - 1, 1:n - 1] = True
    else:
        m[0:n - 1, 1:n - 1, 1:n - 1] = True
    return m


# D3Q7 velocities and weights of Eq. (5) (rest weight 1/4), for callers that
# have no oracle at hand
E7 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
W7 = np.array([0.25] + [0.125] * 6)
