"""Manufactured solution with two exponential layers (Sec. 3.3, eq.
exponential_MMS) and its forcing term, for the discretisation pins.

u(x,y) = X(x) Y(y), X = g (1 - e^{-2x/eps}), g = cos(pi x/2),
                    Y = q (1 - e^{-3y/eps}), q = (1 - y)^3,
f = -eps Lap u - 2 u_x - 3 u_y + u.

For X = g (1 - E), E = e^{-a x/eps}:  -eps X'' - a X' = (1 - E)(-eps g'' - a g')
- 2 a g' E  (the O(1/eps) terms cancel exactly), so f is formed without
catastrophic cancellation.
"""
import numpy as np


def exponential_mms(eps, x, y):
    X, Y = np.meshgrid(x, y)  # [j, i]
    g = np.cos(np.pi * X / 2)
    gp = -(np.pi / 2) * np.sin(np.pi * X / 2)
    gpp = -(np.pi ** 2 / 4) * np.cos(np.pi * X / 2)
    q = (1 - Y) ** 3
    qp = -3 * (1 - Y) ** 2
    qpp = 6 * (1 - Y)
    E = np.exp(-2 * X / eps)
    G = np.exp(-3 * Y / eps)
    XX = g * (1 - E)
    YY = q * (1 - G)
    LX = (1 - E) * (-eps * gpp - 2 * gp) - 4 * gp * E   # -eps X'' - 2 X'
    LY = (1 - G) * (-eps * qpp - 3 * qp) - 6 * qp * G   # -eps Y'' - 3 Y'
    f = YY * LX + XX * LY + XX * YY
    u = XX * YY
    return u[1:-1, 1:-1].ravel(), f[1:-1, 1:-1].ravel()
