"""FP64 oracle of the charge-conserving current deposition (test infrastructure only; the
product path never imports it).

Sec. II.C: the current follows from the change of the particles' charge density over a
step through the continuity equation (Esirkepov's decomposition), so that the field solver
(Sec. II.B, E += dt (curl B - J)) keeps Gauss's law once it holds initially.  Shapes are the
TSC weights of Sec. II.E, node-centred: for a coordinate X in cell units the nearest node is
j = floor(X + 1/2), d = X - j, and the weights of nodes j-1, j, j+1 are
(1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2.

2D grid in the x-y plane (z squeezed), the staggering of the field arrays ([ny][nx], node
(i, j) at (gx0 + i dx, gy0 + j dy)):
    rho at (i, j);  Jx at (i+1/2, j);  Jy at (i, j+1/2);  Jz at (i, j);
periodic in x and y.  A particle of charge Q = q w qscale moving from (xa, ya, za) to
(xb, yb, zb) in one step dt (less than one cell in x and in y) contributes, with S0 / S1
its shapes at the start / end and DS = S1 - S0 on a common 5 x 5 node window:
    Wx = DSx (S0y + DSy/2),   Wy = DSy (S0x + DSx/2),
    Wz = S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3
         (the mean over the step of the product of the linearly interpolated shapes),
    Jx(i+1/2, j) - Jx(i-1/2, j) = -Q Wx(i, j) / (dy dt),
    Jy(i, j+1/2) - Jy(i, j-1/2) = -Q Wy(i, j) / (dx dt),
    Jz(i, j) = Q (zb - za)/dt Wz(i, j) / (dx dy),
the first two summed from the low side of the window.  Since Wx + Wy = S1x S1y - S0x S0y
this gives (rho1 - rho0)/dt + div J = 0 node by node with rho = Q Sx Sy / (dx dy).
"""
from __future__ import annotations

import math

import numpy as np


def _shape5(X: np.ndarray, base: np.ndarray) -> np.ndarray:
    """TSC weights of coordinate X (cell units) on the five nodes base-2 .. base+2."""
    j = np.floor(X + 0.5)
    d = X - j
    out = np.zeros((len(X), 5))
    k = (j - base).astype(np.int64) + 2          # slot of the nearest node
    rows = np.arange(len(X))
    out[rows, k - 1] = 0.5 * (0.5 - d) ** 2
    out[rows, k] = 0.75 - d * d
    out[rows, k + 1] = 0.5 * (0.5 + d) ** 2
    return out


def rho(x, y, w, q, qscale, nx, ny, dx, dy, gx0=0.0, gy0=0.0) -> np.ndarray:
    """Charge density on the nodes [ny][nx]: sum of Q Sx Sy / (dx dy), periodic."""
    X = (np.asarray(x, float) - gx0) / dx
    Y = (np.asarray(y, float) - gy0) / dy
    bx, by = np.floor(X + 0.5), np.floor(Y + 0.5)
    Sx, Sy = _shape5(X, bx), _shape5(Y, by)
    Q = q * np.asarray(w, float) * qscale / (dx * dy)
    out = np.zeros((ny, nx))
    for a in range(5):
        for b in range(5):
            np.add.at(out, (((by + b - 2) % ny).astype(np.int64), ((bx + a - 2) % nx).astype(np.int64)),
                      Q * Sx[:, a] * Sy[:, b])
    return out


def deposit(xa, ya, za, xb, yb, zb, w, q, qscale, dt, nx, ny, dx, dy, gx0=0.0, gy0=0.0):
    """Jx, Jy, Jz ([ny][nx] each) of particles moving from (xa, ya, za) to (xb, yb, zb) over
    dt.  Every displacement must be below one cell in x and in y."""
    xa, ya, za, xb, yb, zb, w = (np.asarray(v, float) for v in (xa, ya, za, xb, yb, zb, w))
    Xa, Ya, Xb, Yb = (xa - gx0) / dx, (ya - gy0) / dy, (xb - gx0) / dx, (yb - gy0) / dy
    if np.any(np.abs(Xb - Xa) >= 1) or np.any(np.abs(Yb - Ya) >= 1):
        raise ValueError("a displacement of one cell or more")
    bx, by = np.floor(Xa + 0.5), np.floor(Ya + 0.5)           # window centred on the start node
    S0x, S1x = _shape5(Xa, bx), _shape5(Xb, bx)
    S0y, S1y = _shape5(Ya, by), _shape5(Yb, by)
    DSx, DSy = S1x - S0x, S1y - S0y
    Q = q * w * qscale
    Jx, Jy, Jz = np.zeros((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
    col = [((bx + a - 2) % nx).astype(np.int64) for a in range(5)]
    row = [((by + b - 2) % ny).astype(np.int64) for b in range(5)]
    vz = (zb - za) / dt
    for b in range(5):
        run = np.zeros(len(Q))
        for a in range(5):
            run = run - Q * DSx[:, a] * (S0y[:, b] + 0.5 * DSy[:, b]) / (dy * dt)
            np.add.at(Jx, (row[b], col[a]), run)
    for a in range(5):
        run = np.zeros(len(Q))
        for b in range(5):
            run = run - Q * DSy[:, b] * (S0x[:, a] + 0.5 * DSx[:, a]) / (dx * dt)
            np.add.at(Jy, (row[b], col[a]), run)
    for a in range(5):
        for b in range(5):
            wz = (S0x[:, a] * S0y[:, b] + 0.5 * DSx[:, a] * S0y[:, b] + 0.5 * S0x[:, a] * DSy[:, b]
                  + DSx[:, a] * DSy[:, b] / 3.0)
            np.add.at(Jz, (row[b], col[a]), Q * vz * wz / (dx * dy))
    return Jx, Jy, Jz


def divergence(Jx, Jy, dx, dy) -> np.ndarray:
    """Discrete divergence of a (Jx, Jy) pair at the nodes (backward differences, periodic)."""
    return (Jx - np.roll(Jx, 1, axis=1)) / dx + (Jy - np.roll(Jy, 1, axis=0)) / dy


def tsc_weights(X: float):
    """(nearest node, [w_{j-1}, w_j, w_{j+1}]) of one coordinate, for brute-force checks."""
    j = math.floor(X + 0.5)
    d = X - j
    return j, [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
