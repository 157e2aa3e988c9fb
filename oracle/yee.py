"""FP64 oracle of the 2D vacuum field solver (test infrastructure only; the product path
never imports it).

Maxwell's curl equations in normalised units on the 2D Yee grid of Sec. II.B (z
squeezed, d/dz = 0), with the staggering of the grid field: array index [j][i] holds
  Ex at (i+1/2, j), Ey at (i, j+1/2), Ez at (i, j),
  Bx at (i, j+1/2), By at (i+1/2, j), Bz at (i+1/2, j+1/2),
periodic in both directions.  One step of dt (leapfrog, Sec. II.F, with B split into two
half steps so that E and B are both known at integer times):
  B -= dt/2 curl E;  E += dt (curl B - J);  B -= dt/2 curl E,
with J = (Jx, Jy, Jz) at the staggering of E and the half-integer time of the step (zero
when no current is given).
The differences are written out with numpy's roll (periodic wrap).
"""
from __future__ import annotations

import numpy as np

EX, EY, EZ, BX, BY, BZ = range(6)


def _dxf(a, dx):
    """forward difference along x: (a[i+1] - a[i]) / dx"""
    return (np.roll(a, -1, axis=1) - a) / dx


def _dxb(a, dx):
    """backward difference along x: (a[i] - a[i-1]) / dx"""
    return (a - np.roll(a, 1, axis=1)) / dx


def _dyf(a, dy):
    return (np.roll(a, -1, axis=0) - a) / dy


def _dyb(a, dy):
    return (a - np.roll(a, 1, axis=0)) / dy


def b_half(F, dx, dy, h):
    """B -= h curl E (h = dt/2):
    Bx(i, j+1/2) -= h dEz/dy;  By(i+1/2, j) += h dEz/dx;
    Bz(i+1/2, j+1/2) -= h (dEy/dx - dEx/dy)."""
    Ex, Ey, Ez = F[EX], F[EY], F[EZ]
    F[BX] = F[BX] - h * _dyf(Ez, dy)
    F[BY] = F[BY] + h * _dxf(Ez, dx)
    F[BZ] = F[BZ] - h * (_dxf(Ey, dx) - _dyf(Ex, dy))


def e_full(F, dx, dy, dt, J=None):
    """E += dt (curl B - J):
    Ex(i+1/2, j) += dt (dBz/dy - Jx);  Ey(i, j+1/2) -= dt (dBz/dx + Jy);
    Ez(i, j) += dt (dBy/dx - dBx/dy - Jz)."""
    Bx, By, Bz = F[BX], F[BY], F[BZ]
    F[EX] = F[EX] + dt * _dyb(Bz, dy)
    F[EY] = F[EY] - dt * _dxb(Bz, dx)
    F[EZ] = F[EZ] + dt * (_dxb(By, dx) - _dyb(Bx, dy))
    if J is not None:
        F[EX] = F[EX] - dt * J[0]
        F[EY] = F[EY] - dt * J[1]
        F[EZ] = F[EZ] - dt * J[2]


def advance(F, dx: float, dy: float, dt: float, steps: int = 1, J=None):
    """Advance the six FP64 arrays F[0..5] (each [ny][nx]) by `steps` steps in place, with
    the current J (three [ny][nx] arrays, held fixed over the steps) if given."""
    for _ in range(steps):
        b_half(F, dx, dy, 0.5 * dt)
        e_full(F, dx, dy, dt, J)
        b_half(F, dx, dy, 0.5 * dt)
    return F


def div_b(F, dx, dy):
    """Discrete divergence of B at the cell centres (i+1/2, j+1/2) (d/dz = 0)."""
    return _dxf(F[BX], dx) + _dyf(F[BY], dy)


def div_e(F, dx, dy):
    """Discrete divergence of E at the nodes (i, j)."""
    return _dxb(F[EX], dx) + _dyb(F[EY], dy)
