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

Open x boundaries (first-order absorbing condition of Mur, with an incoming pulse injected
through x_max): the E update runs as above, then the tangential components Ey, Ez on the
first and last node columns are replaced by the one-way wave condition of the outgoing
(scattered) field, (d/dt - d/dx) E = 0 at x_min and (d/dt + d/dx)(E - E_inc) = 0 at x_max,
discretised between the boundary node and its neighbour over the step:
  E_0^{n+1} = E_1^n + k (E_1^{n+1} - E_0^n),   k = (dt - dx)/(dt + dx),
and at x_max the same for E - E_inc with E_inc the analytic incoming field at each node's
staggered position and time.  The second B half step then sees the corrected E; the
values the periodic wrap leaves in the cells beyond the boundaries never reach the
interior; the components half a cell beyond x_max (Ex, By, Bz of the last column) lie
outside the box and are kept at zero.  y stays periodic.
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


def _incoming(spec, t, x, ys):
    """E of the analytic pulse `spec` at the points (x, y, 0), y in ys, time t: [len(ys)][3]."""
    import oracle                                  # the C oracle's field evaluation
    pts = np.stack([np.full(len(ys), x), np.asarray(ys, float), np.zeros(len(ys))], axis=1)
    return oracle.field_eval_points(spec, t, pts)[0]


def _mur(F, old, dx, dy, dt, bc, t0, t1):
    """Replace Ey, Ez on the first and last node columns (first-order Mur condition; the
    incoming pulse bc['incoming'] enters through x_max)."""
    k = (dt - dx) / (dt + dx)
    ny, nx = F[EY].shape
    for c in (EY, EZ):
        L0, L1, R0, R1 = old[c]
        F[c][:, 0] = L1 + k * (F[c][:, 1] - L0)
        inc = bc.get("incoming")
        if inc is None:
            F[c][:, nx - 1] = R1 + k * (F[c][:, nx - 2] - R0)
            continue
        half = 0.5 if c == EY else 0.0              # Ey at (i, j+1/2), Ez at (i, j)
        ys = bc["gy0"] + (np.arange(ny) + half) * dy
        xN, xM = bc["gx0"] + (nx - 1) * dx, bc["gx0"] + (nx - 2) * dx
        comp = 1 if c == EY else 2
        IN0, IN1 = _incoming(inc, t0, xN, ys)[:, comp], _incoming(inc, t1, xN, ys)[:, comp]
        IM0, IM1 = _incoming(inc, t0, xM, ys)[:, comp], _incoming(inc, t1, xM, ys)[:, comp]
        F[c][:, nx - 1] = IN1 + (R1 - IM0) + k * ((F[c][:, nx - 2] - IM1) - (R0 - IN0))


def advance(F, dx: float, dy: float, dt: float, steps: int = 1, J=None, bc=None):
    """Advance the six FP64 arrays F[0..5] (each [ny][nx]) by `steps` steps in place, with
    the current J (three [ny][nx] arrays, held fixed over the steps) if given.  bc = None
    (periodic) or a dict {'open_x': True, 'incoming': pulse spec or None, 'gx0', 'gy0',
    't0'} for open x boundaries; t0 is the time of F on entry."""
    open_x = bc is not None and bc.get("open_x")
    for n in range(steps):
        if open_x:
            old = {c: (F[c][:, 0].copy(), F[c][:, 1].copy(), F[c][:, -1].copy(), F[c][:, -2].copy())
                   for c in (EY, EZ)}
        b_half(F, dx, dy, 0.5 * dt)
        e_full(F, dx, dy, dt, J)
        if open_x:
            _mur(F, old, dx, dy, dt, bc, bc["t0"] + n * dt, bc["t0"] + (n + 1) * dt)
        b_half(F, dx, dy, 0.5 * dt)
        if open_x:
            for c in (EX, BY, BZ):
                F[c][:, -1] = 0.0
    return F


def energy(F, dx, dy):
    """Field energy (1/2) sum (E^2 + B^2) dx dy over the grid (normalised units)."""
    return 0.5 * sum(float((f * f).sum()) for f in F) * dx * dy


def div_b(F, dx, dy):
    """Discrete divergence of B at the cell centres (i+1/2, j+1/2) (d/dz = 0)."""
    return _dxf(F[BX], dx) + _dyf(F[BY], dy)


def div_e(F, dx, dy):
    """Discrete divergence of E at the nodes (i, j)."""
    return _dxb(F[EX], dx) + _dyb(F[EY], dy)
