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


def parabolic_mms(eps, x, y):
    """One parabolic and one exponential layer (Sec. 3.3, eq. parabolic_MMS):
    -eps Lap u - u_x + u = f with u = X(x) Y(y),
      X = g - (e^{-x/eps} - e^{-1/eps}) / (1 - e^{-1/eps}),  g = cos(pi x/2),
      Y = (1 - e^{-y/sqrt(eps)}) / (1 - e^{-1/sqrt(eps)}) - y^{5/2}.
    The layer term of X solves -eps X'' - X' = 0 exactly, so
    -eps X'' - X' = -eps g'' - g'; and -eps Y'' = e^{-y/sqrt(eps)} /
    (1 - e^{-1/sqrt(eps)}) + (15/4) eps sqrt(y)."""
    X, Y = np.meshgrid(x, y)  # [j, i]
    se = np.sqrt(eps)
    g = np.cos(np.pi * X / 2)
    gp = -(np.pi / 2) * np.sin(np.pi * X / 2)
    gpp = -(np.pi ** 2 / 4) * np.cos(np.pi * X / 2)
    E1, G1 = np.exp(-1.0 / eps), np.exp(-1.0 / se)
    XX = g - (np.exp(-X / eps) - E1) / (1 - E1)
    G = np.exp(-Y / se)
    YY = (1 - G) / (1 - G1) - Y ** 2.5
    LX = -eps * gpp - gp                                  # -eps X'' - X'
    LY = G / (1 - G1) + 3.75 * eps * np.sqrt(Y)           # -eps Y''
    f = LX * YY + XX * LY + XX * YY
    u = XX * YY
    return u[1:-1, 1:-1].ravel(), f[1:-1, 1:-1].ravel()
